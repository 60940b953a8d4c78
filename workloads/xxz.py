"""Spin-1/2 XXZ ring with random fields and complex (phase-twisted) XY bonds.

H = sum_i [ (J_xy/2) (e^{i phi_i} S+_i S-_{i+1} + e^{-i phi_i} S-_i S+_{i+1}) + J_z Sz_i Sz_{i+1} ]
    + sum_i h_i Sz_i,    periodic (site L == site 0), S = sigma/2.

Basis state s is an L-bit integer, bit i set <=> spin i up.  Row s holds its
diagonal (always stored) and one entry per anti-parallel bond i at column
s ^ (1<<i | 1<<(i+1 mod L)); the value is (J_xy/2) e^{+i phi_i} when s has
bit i up and bit i+1 down, otherwise (J_xy/2) e^{-i phi_i}.  nnz = 2^L (1 + L/2).

Draw order from default_rng(seed): h = uniform(-1, 1, L); phi = uniform(0, 2 pi, L);
then v0 = standard_normal(d) + 1j standard_normal(d), normalised.
"""

import numpy as np

from .csr import CSR, random_state


def xxz_nnz(L: int) -> int:
    """Closed form: every row stores its diagonal plus, on average, L/2 anti-parallel bonds."""
    return (2 ** L) * (2 + L) // 2


def xxz_chain(L: int, seed: int, j_xy: float = 1.0, j_z: float = 0.5, with_v0: bool = True,
              n_v0: int = 1):
    """Return (CSR, v0) for the XXZ ring on L >= 3 sites.

    With ``n_v0 > 1`` the second element is a list of n_v0 vectors drawn one
    after the other from the same generator (the first equals the n_v0 == 1 draw).
    """
    if L < 3:
        raise ValueError("L >= 3 required (periodic ring)")
    rng = np.random.default_rng(seed)
    h = rng.uniform(-1.0, 1.0, L)
    phi = rng.uniform(0.0, 2.0 * np.pi, L)
    d = 1 << L
    s = np.arange(d, dtype=np.int64)

    diag = np.zeros(d)
    up = [((s >> i) & 1).astype(bool) for i in range(L)]
    for i in range(L):
        j = (i + 1) % L
        sz_i = np.where(up[i], 0.5, -0.5)
        sz_j = np.where(up[j], 0.5, -0.5)
        diag += j_z * sz_i * sz_j + h[i] * sz_i

    # per-row count of entries: 1 + number of anti-parallel bonds
    counts = np.ones(d, dtype=np.int64)
    for i in range(L):
        counts += up[i] != up[(i + 1) % L]
    row_ptr = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    assert nnz == xxz_nnz(L)

    # Fill unsorted, then sort columns inside every row with one global argsort on (row, col).
    cols = np.empty(nnz, dtype=np.int64)
    vals = np.empty(nnz, dtype=np.complex128)
    fill = row_ptr[:-1].copy()
    cols[fill] = s
    vals[fill] = diag
    fill += 1
    half = 0.5 * j_xy
    for i in range(L):
        j = (i + 1) % L
        anti = up[i] != up[j]
        rows = s[anti]
        pos = fill[anti]
        cols[pos] = rows ^ ((1 << i) | (1 << j))
        vals[pos] = np.where(up[i][anti], half * np.exp(1j * phi[i]), half * np.exp(-1j * phi[i]))
        fill[anti] += 1
    row_of = np.repeat(s, counts)
    order = np.argsort(row_of * d + cols, kind="stable")
    csr = CSR(d, row_ptr.astype(np.int32), cols[order].astype(np.int32),
              np.ascontiguousarray(vals[order]), f"xxz_L{L}_s{seed}")
    if not with_v0:
        return csr, None
    if n_v0 == 1:
        return csr, random_state(rng, d)
    return csr, [random_state(rng, d) for _ in range(n_v0)]


def magnon_sector(L: int, n_up: int) -> np.ndarray:
    """Indices of basis states with exactly n_up spins up (H conserves this number)."""
    s = np.arange(1 << L, dtype=np.int64)
    pop = np.zeros_like(s)
    for i in range(L):
        pop += (s >> i) & 1
    return np.nonzero(pop == n_up)[0]
