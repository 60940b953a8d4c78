"""Open Bose chain built on the device (Sec. "Creation of Hamiltonian Matrix": number-state
basis of fixed total occupation, eqs. basisState, totalOccupationNumber, findIndices).

Small and medium chains: row pointers, columns and hop values are bitwise those of the host
workload builder (explicit basis + sorted-key lookup table); the diagonal agrees to rounding
(the host sums it with a matrix-vector product).  A large chain: sampled rows against a per-row
reference written here from the operator definitions, with basis indices from a direct count of
the states that precede (no closed form shared with the device).  Evolution on a device-built
chain matches the oracle."""

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import announce, lib, to_dev, to_host

pytestmark = pytest.mark.gpu

# (K modes, N bosons): single mode, no bosons, one boson, wide and deep chains, K > 32 (more
# entry slots than lanes; the host builder's packed keys limit these to N = 1), K = 64 (128
# slots), several rows per workgroup with a ragged tail
CASES = [(1, 0), (1, 4), (2, 0), (2, 9), (3, 1), (3, 5), (6, 4), (8, 5), (12, 3), (4, 12),
         (40, 1), (64, 1), (10, 9), (16, 6)]


def params(K, seed):
    return W.bose_chain_params(np.random.default_rng(seed), K)


def check_against_host(te, K, N, seed):
    Hh, _ = W.bosonic_chain(K, N, seed, with_v0=False)
    U, a = params(K, seed)
    h = te.te_hamiltonian_create_bose_chain(U, a, N)
    assert (h.dim, h.nnz) == (Hh.dim, Hh.nnz) == (math.comb(N + K - 1, K - 1), Hh.nnz)
    rp, ci, va = te.te_hamiltonian_copy_csr(h)
    assert np.array_equal(rp, Hh.row_ptr) and np.array_equal(ci, Hh.col)
    rows = np.repeat(np.arange(Hh.dim), np.diff(Hh.row_ptr))
    off = Hh.col != rows
    assert np.array_equal(va[off].view(np.float64), Hh.val[off].view(np.float64))
    occ = W.fock_basis(K, N).astype(np.float64)
    scale = (occ * np.abs(occ - 1.0)) @ U  # sum of the magnitudes of the diagonal's terms
    assert np.all(np.abs(va[~off].real - Hh.val[~off].real) <= 4 * np.finfo(float).eps * scale)
    assert not np.any(va[~off].imag)
    return h, Hh


@pytest.mark.parametrize("K,N", CASES)
def test_device_build_matches_the_host_build(K, N):
    announce(f"bose chain build K={K} N={N}")
    te = lib()
    h, _ = check_against_host(te, K, N, seed=100 + K + N)
    assert h.real_values == (K == 1 or N == 0)  # a matrix with hops has complex entries
    h.destroy()


def test_real_hops_keep_real_entries():
    announce("bose chain, real hops")
    te = lib()
    K, N = 7, 5
    U, a = params(K, 9)
    h = te.te_hamiltonian_create_bose_chain(U, np.abs(a), N)
    hc = te.te_hamiltonian_create_bose_chain(U, np.abs(a), N, store_complex=True)
    assert h.real_values and not hc.real_values and h.norm1 == hc.norm1
    r1, c1, v1 = te.te_hamiltonian_copy_csr(h)
    r2, c2, v2 = te.te_hamiltonian_copy_csr(hc)
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2) and np.array_equal(v1, v2)
    h.destroy()
    hc.destroy()


def test_evolution_on_the_device_build_matches_oracle():
    announce("bose chain evolution")
    te = lib()
    K, N = 8, 5
    h, Hh = check_against_host(te, K, N, seed=4)
    v0 = W.random_state(np.random.default_rng(5), Hh.dim)
    v, res = te.te_evolve(h, to_dev(v0), 3.0, 1e-8, 40)
    ro = O.evolve(Hh, v0, 3.0, 1e-8, 40)
    assert np.linalg.norm(to_host(v) - ro.v) <= 2e-8 + 1e-12 and res.err_bound <= 1e-8
    h.destroy()


def _rank(n, N):
    """Index of occupation tuple n in descending lexicographic order: a direct count of the
    tuples that agree before mode i and hold more bosons there, summed over the modes."""
    K, R, rank = len(n), N, 0
    for i in range(K - 1):
        for v in range(n[i] + 1, R + 1):
            rest, modes = R - v, K - i - 1  # compositions of `rest` into `modes` parts
            rank += math.comb(rest + modes - 1, modes - 1)
        R -= n[i]
    return rank


def _row_reference(n, N, U, a):
    """Entries (col, value) of the row of state n from the operator definitions."""
    K = len(n)
    out = {_rank(n, N): sum(U[k] * n[k] * (n[k] - 1.0) for k in range(K))}
    for k in range(K - 1):
        if n[k] > 0:  # a_k b_k^+ b_{k+1} applied to the state with one boson moved to k + 1
            s = list(n)
            s[k] -= 1
            s[k + 1] += 1
            out[_rank(s, N)] = a[k] * np.sqrt(s[k + 1] * (s[k] + 1.0))
        if n[k + 1] > 0:  # conj(a_k) b_{k+1}^+ b_k applied to the state with one boson moved to k
            s = list(n)
            s[k] += 1
            s[k + 1] -= 1
            out[_rank(s, N)] = np.conj(a[k]) * np.sqrt(s[k] * (s[k + 1] + 1.0))
    cols = sorted(out)
    return np.array(cols, dtype=np.int64), np.array([out[c] for c in cols], dtype=np.complex128)


@pytest.mark.parametrize("K,N", [(30, 6), (33, 4), (64, 3)])
def test_sampled_rows(K, N):
    """Chains beyond the host builder: K = 30, N = 6 (d = 1,623,160); K > 32 with N > 1."""
    announce(f"bose chain K={K} N={N}, sampled rows")
    te = lib()
    U, a = params(K, 21)
    h = te.te_hamiltonian_create_bose_chain(U, a, N)
    assert h.dim == math.comb(N + K - 1, K - 1)
    rp, ci, va = te.te_hamiltonian_copy_csr(h)
    assert rp[0] == 0 and rp[-1] == h.nnz and np.all(np.diff(rp) >= 1)
    rng = np.random.default_rng(8)
    states = [[N] + [0] * (K - 1), [0] * (K - 1) + [N], [1] * N + [0] * (K - N)]
    for _ in range(60):  # random compositions of N into K parts
        cuts = np.sort(rng.integers(0, N + 1, K - 1))
        states.append(list(np.diff(np.concatenate([[0], cuts, [N]]))))
    for n in states:
        r = _rank(n, N)
        cols, vals = _row_reference([int(x) for x in n], N, U, a)
        lo, hi = rp[r], rp[r + 1]
        assert np.array_equal(ci[lo:hi], cols), n
        d = cols == r
        assert np.array_equal(va[lo:hi][~d], vals[~d]), n
        assert abs(va[lo:hi][d][0] - vals[d][0]) <= 1e-13 * max(1.0, abs(vals[d][0])), n
    assert _rank(states[0], N) == 0 and _rank(states[1], N) == h.dim - 1
    h.destroy()


@pytest.mark.parametrize("K,N,status", [(0, 3, "TE_ERR_INVALID_ARG"), (65, 1, "TE_ERR_INVALID_ARG"),
                                        (4, -1, "TE_ERR_INVALID_ARG"), (2, 70000, "TE_ERR_INVALID_ARG"),
                                        (64, 12, "TE_ERR_UNSUPPORTED")])
def test_arguments_out_of_range(K, N, status):
    announce(f"bose chain arguments K={K} N={N}")
    te = lib()
    U = np.ones(max(K, 1))
    a = np.ones(max(K - 1, 0), dtype=np.complex128)
    with pytest.raises(te.TEError) as e:
        te.te_hamiltonian_create_bose_chain(U[:K] if K else U[:0], a, N)
    assert e.value.status == getattr(te, status)


def test_non_finite_parameter():
    announce("bose chain, non-finite parameter")
    te = lib()
    U, a = params(5, 2)
    a[2] = np.nan
    with pytest.raises(te.TEError) as e:
        te.te_hamiltonian_create_bose_chain(U, a, 3)
    assert e.value.status == te.TE_ERR_INVALID_ARG
