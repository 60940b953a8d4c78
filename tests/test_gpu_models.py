"""The paper's exemplary Hamiltonian (eq. fullHamiltonianSimple) built on the device.

Small and medium parameter sets: the device CSR (row pointers, columns, values) is bitwise the
one the host workload builder assembles from its explicit basis and lookup table, and the
evolution on it matches the oracle.  The paper's own size (d = 1,565,904): structure, the
closed-form row lengths, and sampled rows against a per-row reference written here from the
operator definitions (ranks of the qubit configurations by direct enumeration)."""

import itertools
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import announce, lib, to_dev, to_host
from workloads import memory_burden as MB

pytestmark = pytest.mark.gpu

CASES = [
    {},  # the paper's Fig. 1 system, d = 588
    dict(K=5, Kp=5, N0=8, Nm=3, eps_m=1.7, Nc=11.0, dNc=3.5, C0=0.7, Cm=1.3),
    dict(K=3, Kp=0, N0=0, Nm=1),  # no second memory kind, no a_0 / b_0 dynamics
    dict(K=6, Kp=2, N0=3, Nm=6),
    dict(K=4, Kp=3, N0=5, Nm=0),  # empty memory: diagonal + C_0 hopping only
]


def build_both(te, params):
    Hh, v0, _ = MB.memory_burden_model(**params)
    h, idx = te.te_hamiltonian_create_memory_burden(**params)
    return Hh, v0, h, idx


@pytest.mark.parametrize("params", CASES)
def test_device_build_is_bitwise_the_host_build(params):
    announce(f"memory burden build {params}")
    te = lib()
    Hh, v0, h, idx = build_both(te, params)
    assert (h.dim, h.nnz) == (Hh.dim, Hh.nnz) and h.real_values
    rp, ci, va = te.te_hamiltonian_copy_csr(h)
    assert np.array_equal(rp, Hh.row_ptr) and np.array_equal(ci, Hh.col)
    assert np.array_equal(va.view(np.float64), Hh.val.view(np.float64))
    assert idx == int(np.flatnonzero(v0)[0])
    hr = te.te_hamiltonian_create(Hh.row_ptr, Hh.col, Hh.val)
    assert hr.norm1 == h.norm1
    hr.destroy()
    h.destroy()


def test_evolution_on_the_device_build_matches_oracle():
    announce("memory burden evolution")
    te = lib()
    params = CASES[1]
    Hh, v0, h, idx = build_both(te, params)
    v, res = te.te_evolve(h, to_dev(v0), 6.0, 1e-8, 40)
    ro = O.evolve(Hh, v0, 6.0, 1e-8, 40)
    assert np.linalg.norm(to_host(v) - ro.v) <= 2e-8 + 1e-12 and res.err_bound <= 1e-8
    h.destroy()


def _rank(bits, n):
    """Descending-lexicographic rank among tuples with the same number of ones (direct count of
    the tuples that precede: at each 0 with r ones left, those placing a 1 there)."""
    rank, r = 0, sum(bits)
    for i, b in enumerate(bits):
        if r == 0:
            break
        if b:
            r -= 1
        else:
            rank += math.comb(n - 1 - i, r - 1)
    return rank


def _row_reference(p, r, configs, index_of):
    """Entries (col, value) of row r from the operator definitions."""
    K, Kp, N0, Nm = p["K"], p["Kp"], p["N0"], p["Nm"]
    n, C = K + Kp, len(configs)
    i0, i1 = divmod(r, C)
    n0, m0 = N0 - i0, i0
    bits = configs[i1]
    nk, nkp = sum(bits[:K]), sum(bits[K:])
    out = {r: p["eps_m"] * (1.0 - n0 / p["Nc"]) * nk + p["eps_m"] * (1.0 - n0 / (p["Nc"] - p["dNc"])) * nkp}

    def amp(u, v):
        a, b = min(u, v), max(u, v)
        if b < K:
            return p["Cm"] * MB._f(2, a + 1, b + 1, K)
        if a >= K:
            return p["Cm"] * MB._f(3, a - K + 1, b - K + 1, K)
        return p["Cm"] * MB._f(1, a + 1, b - K + 1, K)

    for u in range(n):
        for v in range(n):
            if bits[u] == 1 and bits[v] == 0:
                src = list(bits)
                src[u], src[v] = 0, 1
                out[i0 * C + index_of[tuple(src)]] = amp(u, v) * np.sqrt(1 * (0 + 1.0))
    if n0 > 0:  # a_0^+ b_0 acting on (n_0 - 1, m_0 + 1)
        out[r + C] = p["C0"] * np.sqrt((m0 + 1) * ((n0 - 1) + 1.0))
    if n0 < N0:  # b_0^+ a_0 acting on (n_0 + 1, m_0 - 1)
        out[r - C] = p["C0"] * np.sqrt((n0 + 1) * ((m0 - 1) + 1.0))
    cols = sorted(out)
    return np.array(cols, dtype=np.int64), np.array([out[c] for c in cols])


def test_papers_size_built_on_the_device():
    """K = K' = 10, N_0 = 100, N_m = 5 (Sec. "Analysis of Performance"): d = 1,565,904."""
    announce("memory burden, paper's size")
    te = lib()
    params = dict(MB.DEFAULTS, K=10, Kp=10, N0=100, Nm=5, Nc=100.0)
    h, idx = te.te_hamiltonian_create_memory_burden(**{k: params[k] for k in
                                                       ("K", "Kp", "N0", "Nm", "eps_m", "Nc", "dNc", "C0", "Cm")})
    n, Nm, N0 = 20, 5, 100
    C = math.comb(n, Nm)
    assert h.dim == 1565904 == (N0 + 1) * C and h.real_values and idx == 0
    Q = Nm * (n - Nm)
    assert h.nnz == C * ((N0 + 1) * (1 + Q) + 2 * N0)
    rp, ci, va = te.te_hamiltonian_copy_csr(h)
    lens = np.diff(rp.astype(np.int64)).reshape(N0 + 1, C)
    assert np.all(lens[0] == 2 + Q) and np.all(lens[N0] == 2 + Q) and np.all(lens[1:N0] == 3 + Q)
    # configurations in descending lexicographic order, with their ranks
    configs = [tuple(1 if i in ones else 0 for i in range(n)) for ones in itertools.combinations(range(n), Nm)]
    configs.sort(reverse=True)
    index_of = {c: k for k, c in enumerate(configs)}
    assert all(_rank(c, n) == k for k, c in enumerate(configs[:200]))
    rng = np.random.default_rng(3)
    rows = [0, 1, C - 1, C, h.dim - 1] + list(rng.integers(0, h.dim, 40))
    for r in rows:
        cols, vals = _row_reference(params, int(r), configs, index_of)
        a, b = rp[r], rp[r + 1]
        assert np.array_equal(ci[a:b], cols), r
        assert np.array_equal(va[a:b].real, vals) and not np.any(va[a:b].imag), r
    h.destroy()
