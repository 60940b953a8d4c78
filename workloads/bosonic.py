"""Bosonic chain in a number-eigenstate (Fock) basis with a fixed total occupation.

Basis (paper, Sec. "Creation of Hamiltonian Matrix", eqs. basisState and
totalOccupationNumber): all occupation tuples (n_1..n_K) with sum N, optionally
with a per-mode maximal occupation.  The fixed enumeration ``ind`` is descending
lexicographic order starting from (N, 0, ..., 0).  Its inverse ``ind^-1`` (eq.
findIndices) is a lookup table keyed by the packed tuple (one bit field per mode); the
paper keeps this map in a hash table, here it is a sorted key array searched
with ``numpy.searchsorted`` (same map, constant-factor different).

Model (open chain, K-1 bonds):
  H = sum_k ( a_k b+_k b_{k+1} + conj(a_k) b+_{k+1} b_k ) + sum_k U_k n_k (n_k - 1),
with a_k = r_k e^{i theta_k}.  The diagonal is always stored.

Draw order from default_rng(seed): r = uniform(0.5, 1.5, K-1);
theta = uniform(0, 2 pi, K-1); U = uniform(0, 2, K); then v0 (complex normal on
every basis state, normalised).
"""

from functools import lru_cache
from math import comb

import numpy as np

from .csr import from_triplets, random_state


def fock_dim(K: int, N: int) -> int:
    """Number of ways to put N bosons in K modes: C(N+K-1, K-1)."""
    return comb(N + K - 1, K - 1)


def capped_fock_basis(caps, N: int) -> np.ndarray:
    """All tuples with 0 <= n_k <= caps[k] and sum N, in descending lexicographic order."""
    caps = tuple(int(c) for c in caps)
    K = len(caps)
    suffix_cap = [0] * (K + 1)
    for k in range(K - 1, -1, -1):
        suffix_cap[k] = suffix_cap[k + 1] + caps[k]

    @lru_cache(maxsize=None)
    def rec(k: int, n: int):
        if k == K - 1:
            if n <= caps[k]:
                return np.array([[n]], dtype=np.uint8)
            return np.zeros((0, 1), dtype=np.uint8)
        blocks = []
        for first in range(min(n, caps[k]), -1, -1):
            if n - first > suffix_cap[k + 1]:
                break
            rest = rec(k + 1, n - first)
            if rest.shape[0]:
                head = np.full((rest.shape[0], 1), first, dtype=np.uint8)
                blocks.append(np.hstack([head, rest]))
        if not blocks:
            return np.zeros((0, K - k), dtype=np.uint8)
        return np.vstack(blocks)

    if K == 0:
        raise ValueError("at least one mode")
    return rec(0, N)


def fock_basis(K: int, N: int) -> np.ndarray:
    return capped_fock_basis([N] * K, N)


def field_widths(basis: np.ndarray):
    """Bits per mode so that every occupation seen in the basis fits its field."""
    top = basis.max(axis=0) if basis.shape[0] else np.zeros(basis.shape[1], dtype=np.uint8)
    return [max(1, int(t).bit_length()) for t in top]


def pack(occ: np.ndarray, widths) -> np.ndarray:
    """Pack occupation rows into uint64 keys, mode 0 most significant."""
    if sum(widths) > 64:
        raise ValueError("occupation tuple does not fit a 64-bit key")
    key = np.zeros(occ.shape[0], dtype=np.uint64)
    for k, w in enumerate(widths):
        key = (key << np.uint64(w)) | occ[:, k].astype(np.uint64)
    return key


class FockIndex:
    """ind^-1: occupation tuple -> basis index, for a basis in descending lex order."""

    def __init__(self, basis: np.ndarray):
        self.widths = field_widths(basis)
        self.top = basis.max(axis=0).astype(np.int64)
        keys = pack(basis, self.widths)
        if keys.size > 1 and not np.all(keys[:-1] > keys[1:]):
            raise ValueError("basis must be strictly descending")
        self.asc = keys[::-1].copy()
        self.d = keys.size

    def lookup(self, occ: np.ndarray) -> np.ndarray:
        if occ.shape[0] and np.any(occ.astype(np.int64) > self.top):
            raise KeyError("state outside the basis")
        keys = pack(occ, self.widths)
        pos = np.searchsorted(self.asc, keys)
        pos_c = np.minimum(pos, self.d - 1)
        if not np.all(self.asc[pos_c] == keys):
            raise KeyError("state outside the basis")
        return (self.d - 1 - pos_c).astype(np.int64)


def hopping_triplets(basis, index, src_mode, dst_mode, amp, caps=None):
    """Entries of amp * b+_dst b_src: H[target, source] for every admissible source."""
    n_src = basis[:, src_mode].astype(np.int64)
    n_dst = basis[:, dst_mode].astype(np.int64)
    ok = n_src >= 1
    if caps is not None:
        ok &= n_dst + 1 <= caps[dst_mode]
    source = np.nonzero(ok)[0]
    target_occ = basis[source].copy()
    target_occ[:, src_mode] -= 1
    target_occ[:, dst_mode] += 1
    target = index.lookup(target_occ)
    value = amp * np.sqrt(n_src[source] * (n_dst[source] + 1.0))
    return target, source, value


def bose_chain_params(rng: np.random.Generator, K: int):
    """(U, a) of the chain, drawn in the documented order."""
    r = rng.uniform(0.5, 1.5, K - 1)
    theta = rng.uniform(0.0, 2.0 * np.pi, K - 1)
    U = rng.uniform(0.0, 2.0, K)
    return U, r * np.exp(1j * theta)


def bosonic_chain(K: int, N: int, seed: int, with_v0: bool = True):
    """Return (CSR, v0) for the complex-hopping Bose chain with on-site interaction."""
    rng = np.random.default_rng(seed)
    U, a = bose_chain_params(rng, K)

    basis = fock_basis(K, N)
    d = basis.shape[0]
    index = FockIndex(basis)
    occ = basis.astype(np.float64)
    diag = (occ * (occ - 1.0)) @ U

    rows = [np.arange(d, dtype=np.int64)]
    cols = [np.arange(d, dtype=np.int64)]
    vals = [diag.astype(np.complex128)]
    for k in range(K - 1):
        # a_k b+_k b_{k+1}: a boson moves from mode k+1 to mode k
        t, s, v = hopping_triplets(basis, index, k + 1, k, a[k])
        rows.append(t); cols.append(s); vals.append(v)
        # conj(a_k) b+_{k+1} b_k: a boson moves from mode k to mode k+1
        t, s, v = hopping_triplets(basis, index, k, k + 1, np.conj(a[k]))
        rows.append(t); cols.append(s); vals.append(v)
    csr = from_triplets(d, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                        f"bose_K{K}_N{N}_s{seed}")
    v0 = random_state(rng, d) if with_v0 else None
    return csr, v0
