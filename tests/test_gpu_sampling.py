"""Intermediate-time sampling (te_evolve_sampled) through the C ABI against the oracle's
sampling, exact evolutions and conserved observables.  Bar: every sampled state within
2 tol + 1e-12 of the oracle's and within its reported bound of the exact state; observables
within 2 max|D| (2 tol) + 1e-12 of the oracle's."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu


def sz_diagonal(L):
    return np.array([0.5 * (2 * bin(x).count("1") - L) for x in range(1 << L)], dtype=np.float64)


def dev_f64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("L,m,n_times", [(10, 30, 23), (10, 10, 200), (12, 40, 7)])
def test_sampled_states_match_oracle_and_exact(L, m, n_times):
    announce(f"sampling L={L} m={m} n={n_times}")
    te = lib()
    H, v0 = W.xxz_chain(L, seed=L + 70)
    t, tol = 10.0, 1e-8
    ts = np.linspace(0.0, t, n_times)
    with hamiltonian(H) as h:
        x = to_dev(v0)
        out, res, states, _, bounds = te.te_evolve_sampled(h, x, t, tol, m, ts)
        plain, pres = te.te_evolve(h, x, t, tol, m)
        assert bool((out == plain).all()) and res.steps == pres.steps  # sampling changes nothing else
        S = to_host(states)
    ro = O.evolve(H, v0, t, tol, m, sample_times=ts)
    assert np.all(np.diff(bounds) >= 0) and bounds[-1] == pytest.approx(res.err_bound, rel=1e-14)
    assert np.array_equal(S[-1], to_host(out))
    assert np.linalg.norm(S[0] - v0) <= 1e-13
    check_exact = L <= 10
    for i, ti in enumerate(ts):
        assert np.linalg.norm(S[i] - ro.samples[i]) <= 2 * tol + 1e-12, (i, ti)
        if check_exact:
            assert np.linalg.norm(S[i] - dense_evolve(H, v0, ti)) <= bounds[i] * (1 + 1e-3) + 1e-12


def test_observables_without_states():
    announce("sampling observables")
    te = lib()
    L = 10
    H, v0 = W.xxz_chain(L, seed=81)
    sz = sz_diagonal(L)
    site0 = np.array([0.5 if (x & 1) else -0.5 for x in range(1 << L)])  # S^z of site 0
    D = np.stack([sz, site0])
    ts = np.linspace(0.0, 15.0, 31)
    with hamiltonian(H) as h:
        _, res, states, obs, bounds = te.te_evolve_sampled(h, to_dev(v0), 15.0, 1e-8, 30, ts, states=False,
                                                           obs=dev_f64(D))
    assert states is None and obs.shape == (31, 2)
    ro = O.evolve(H, v0, 15.0, 1e-8, 30, sample_times=ts)
    m0 = np.vdot(v0, sz * v0).real
    for i in range(ts.size):
        v = ro.samples[i]
        for o in range(2):
            want = np.vdot(v, D[o] * v).real
            assert abs(obs[i, o] - want) <= 2 * np.abs(D[o]).max() * 2e-8 + 1e-12, (i, o)
        assert abs(obs[i, 0] - m0) <= 2 * (L / 2) * bounds[i] * 1.01 + 1e-12  # conserved magnetisation
    assert np.ptp(obs[:, 1]) > 1e-3  # the single-site observable moves


def test_bose_mode_occupation():
    announce("sampling bose")
    te = lib()
    K = N = 6
    H, v0 = W.bosonic_chain(K, N, seed=82)
    basis = W.fock_basis(K, N).astype(np.float64)
    D = np.ascontiguousarray(basis.T)  # n_k for every mode k
    ts = np.linspace(0.0, 5.0, 11)
    with hamiltonian(H) as h:
        _, res, _, obs, bounds = te.te_evolve_sampled(h, to_dev(v0), 5.0, 1e-9, 40, ts, states=False,
                                                      obs=dev_f64(D))
    ro = O.evolve(H, v0, 5.0, 1e-9, 40, sample_times=ts)
    for i in range(ts.size):
        v = ro.samples[i]
        want = np.array([np.vdot(v, D[k] * v).real for k in range(K)])
        assert np.abs(obs[i] - want).max() <= 2 * N * 2e-9 + 1e-12
        assert abs(obs[i].sum() - N) <= 2 * N * bounds[i] * 1.01 + 1e-11  # total number


def test_degenerate_cases():
    announce("sampling degenerate")
    te = lib()
    import torch
    H, v0 = W.xxz_chain(8, seed=83)
    sz = sz_diagonal(8)
    with hamiltonian(H) as h:
        x = to_dev(v0)
        # t = 0: every sample is v0
        out, res, st, obs, b = te.te_evolve_sampled(h, x, 0.0, 1e-8, 20, [0.0, 0.0], obs=dev_f64(sz[None, :]))
        assert bool((st[0] == x).all()) and bool((st[1] == x).all()) and np.all(b == 0)
        assert obs[0, 0] == pytest.approx(np.vdot(v0, sz * v0).real, abs=1e-13)
        # zero vector: zero samples, zero bound
        z = torch.zeros_like(x)
        out, res, st, obs, b = te.te_evolve_sampled(h, z, 3.0, 1e-8, 20, [0.0, 1.0, 3.0], obs=dev_f64(sz[None, :]))
        assert float(st.abs().max()) == 0.0 and np.all(obs == 0) and np.all(b == 0) and res.err_bound == 0
        # invalid times
        for bad in ([1.0, 0.5], [-0.5], [0.0, 3.5]):
            with pytest.raises(te.TEError) as ei:
                te.te_evolve_sampled(h, x, 3.0, 1e-8, 20, bad)
            assert ei.value.status == te.TE_ERR_INVALID_ARG
