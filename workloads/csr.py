"""A plain host-side CSR container (int32 indices, complex128 values)."""

from dataclasses import dataclass

import math

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix in compressed-sparse-row form.

    ``row_ptr`` has ``dim + 1`` int32 entries, ``col`` and ``val`` have ``nnz``
    entries; columns are sorted inside every row and the diagonal is always
    stored (possibly as an explicit zero).
    """

    dim: int
    row_ptr: np.ndarray  # int32 [dim + 1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # complex128 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.dim, self.dim))

    def negated(self) -> "CSR":
        """The matrix -H (same pattern), used for forward-backward evolution."""
        return CSR(self.dim, self.row_ptr, self.col, -self.val, self.name + "_neg")

    def norm1(self) -> float:
        """max_j sum_i |H_ij| (the 1-norm)."""
        colsum = np.zeros(self.dim)
        np.add.at(colsum, self.col, np.abs(self.val))
        return float(colsum.max()) if self.dim else 0.0


def from_triplets(dim: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, name: str = "") -> CSR:
    """Build a CSR with sorted columns from (row, col, value) triplets without duplicates."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * dim + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) entries")
    rows = rows[order]
    counts = np.bincount(rows, minlength=dim)
    row_ptr = np.zeros(dim + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(dim, row_ptr.astype(np.int32), cols[order].astype(np.int32),
               np.ascontiguousarray(np.asarray(vals, dtype=np.complex128)[order]), name)


def random_state(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Complex standard-normal vector, normalised to unit 2-norm.

    The squared norm is summed by NumPy's own pairwise summation (no BLAS call), so the vector is
    the same bits for every BLAS thread count (a threaded BLAS dot product sums in an order that
    depends on the number of threads)."""
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    nrm = math.sqrt(float(np.sum(v.real * v.real)) + float(np.sum(v.imag * v.imag)))
    return v / nrm
