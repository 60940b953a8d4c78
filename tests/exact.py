"""Exact references for small problems: dense or block-diagonal eigendecomposition of H.

These are test helpers (not the oracle): they compute exp(-iHt) v through numpy.linalg.eigh,
the textbook route, so the oracle's Krylov result can be pinned against them.
"""

import hashlib

import numpy as np

_EIGH = {}  # digest of a dense matrix -> its eigendecomposition (the last few matrices)


def _eigh(A):
    key = hashlib.sha1(np.ascontiguousarray(A).tobytes()).hexdigest()
    if key not in _EIGH:
        if len(_EIGH) >= 4:
            _EIGH.pop(next(iter(_EIGH)))
        _EIGH[key] = np.linalg.eigh(A)
    return _EIGH[key]


def dense_evolve(H, v0, t):
    A = H.to_scipy().toarray() if hasattr(H, "to_scipy") else np.asarray(H)
    lam, U = _eigh(A)
    return U @ (np.exp(-1j * lam * t) * (U.conj().T @ v0))


def sector_evolve(H, v0, t, sectors):
    """exp(-iHt) v0 for an H that is block diagonal on the given index sets."""
    A = H.to_scipy()
    out = np.zeros_like(v0)
    for idx in sectors:
        if not np.any(v0[idx]):
            continue
        block = A[idx][:, idx].toarray()
        lam, U = np.linalg.eigh(block)
        out[idx] = U @ (np.exp(-1j * lam * t) * (U.conj().T @ v0[idx]))
    return out


def xxz_sectors(L):
    s = np.arange(1 << L)
    pop = np.zeros_like(s)
    for i in range(L):
        pop += (s >> i) & 1
    return [np.nonzero(pop == n)[0] for n in range(L + 1)]


def random_hermitian_csr(d, density, seed, scale=1.0):
    import scipy.sparse as sp
    from workloads.csr import from_triplets
    rng = np.random.default_rng(seed)
    R = sp.random(d, d, density=density, random_state=rng, format="coo")
    vals = (rng.standard_normal(R.nnz) + 1j * rng.standard_normal(R.nnz)) * scale
    A = sp.coo_matrix((vals, (R.row, R.col)), shape=(d, d)).tocsr()
    A = A + A.conj().T + sp.diags(rng.uniform(-1, 1, d) * scale)
    A = A.tocoo()
    A.sum_duplicates()
    return from_triplets(d, A.row, A.col, A.data, f"rand_d{d}_s{seed}")


def few_values_hermitian(d, density, seed, n_values):
    """A random Hermitian pattern whose entries take n_values values (and their conjugates): too
    many (column - row, value) pairs to pack, few values."""
    from workloads.csr import CSR
    R = random_hermitian_csr(d, density, seed)
    rng = np.random.default_rng(seed + 1)
    table = rng.standard_normal(n_values) + 1j * rng.standard_normal(n_values)
    rows = np.repeat(np.arange(d), np.diff(R.row_ptr)).astype(np.int64)
    col = R.col.astype(np.int64)
    lo, hi = np.minimum(rows, col), np.maximum(rows, col)
    mixed = ((lo.astype(np.uint64) * np.uint64(0x9E3779B1) + hi.astype(np.uint64)) * np.uint64(0x85EBCA6B)) >> np.uint64(13)
    v = table[(mixed % np.uint64(n_values)).astype(np.int64)]
    v = np.where(rows < col, v, np.conj(v))
    v = np.where(rows == col, v.real + 0j, v)
    return CSR(d, R.row_ptr, R.col, np.ascontiguousarray(v), f"few_values_{n_values}")
