"""Pins for the oracle's intermediate-time sampling (second remark after Alg. 1: inside the step
holding t_s, v(t_s) = V exp(M (t_s - t_now)) e_1): states against exact evolutions, conserved
diagonal observables, the end points, and that sampling leaves the evolution itself unchanged."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr


def sz_diagonal(L):
    s = np.arange(1 << L)
    return np.array([0.5 * (2 * bin(x).count("1") - L) for x in s], dtype=np.float64)


@pytest.mark.parametrize("case", ["rand", "xxz9", "xxz9_m10"])
def test_samples_within_bound_of_exact(case):
    if case == "rand":
        H = random_hermitian_csr(300, 0.02, 7)
        v0 = W.random_state(np.random.default_rng(8), 300)
        t, tol, m = 4.0, 1e-9, 20
    else:
        H, v0 = W.xxz_chain(9, seed=9)
        t, tol, m = 10.0, 1e-8, (10 if case.endswith("m10") else 30)
    ts = np.linspace(0.0, t, 23)
    res = O.evolve(H, v0, t, tol, m, sample_times=ts)
    assert res.samples.shape == (ts.size, H.dim)
    assert np.all(np.diff(res.sample_bounds) >= 0) and res.sample_bounds[-1] == res.err_bound
    for i, ti in enumerate(ts):
        err = np.linalg.norm(res.samples[i] - dense_evolve(H, v0, ti))
        assert err <= res.sample_bounds[i] * (1 + 1e-3) + 1e-13, (ti, err, res.sample_bounds[i])


def test_end_points_and_unchanged_evolution():
    H, v0 = W.xxz_chain(8, seed=3)
    ts = [0.0, 0.0, 1.7, 5.0, 5.0]
    res = O.evolve(H, v0, 5.0, 1e-9, 20, sample_times=ts)
    plain = O.evolve(H, v0, 5.0, 1e-9, 20)
    assert np.array_equal(res.v, plain.v) and res.steps == plain.steps
    assert np.array_equal(res.samples[3], res.v) and np.array_equal(res.samples[4], res.v)
    assert np.linalg.norm(res.samples[0] - v0) <= 1e-14
    assert np.array_equal(res.samples[0], res.samples[1])


def test_magnetisation_is_conserved_at_every_sample():
    L = 10
    H, v0 = W.xxz_chain(L, seed=12)
    sz = sz_diagonal(L)
    ts = np.linspace(0.0, 20.0, 41)
    res = O.evolve(H, v0, 20.0, 1e-8, 30, sample_times=ts)
    m0 = np.vdot(v0, sz * v0).real
    for i in range(ts.size):
        v = res.samples[i]
        mi = np.vdot(v, sz * v).real
        # <v|D|v> moves by at most 2 ||D|| ||v|| err + ||D|| err^2 under an error of norm err
        assert abs(mi - m0) <= 2 * (L / 2) * res.sample_bounds[i] * 1.01 + 1e-12


def test_mode_occupation_in_the_bose_chain():
    # <n_0>(t_s), the occupation of the first mode (the paper's example observables are such
    # number operators), against the exact evolution; rows of the basis are the CSR rows
    K = N = 5
    H, v0 = W.bosonic_chain(K, N, seed=13)
    n0 = W.fock_basis(K, N)[:, 0].astype(np.float64)
    ts = np.linspace(0.0, 6.0, 13)
    res = O.evolve(H, v0, 6.0, 1e-9, 30, sample_times=ts)
    moved = False
    for i, ti in enumerate(ts):
        v, ex = res.samples[i], dense_evolve(H, v0, ti)
        got, want = np.vdot(v, n0 * v).real, np.vdot(ex, n0 * ex).real
        assert abs(got - want) <= 2 * N * res.sample_bounds[i] * 1.01 + 1e-12
        moved |= abs(want - np.vdot(v0, n0 * v0).real) > 1e-3
    assert moved  # the observable is not trivially constant


def test_invalid_sample_times():
    H, v0 = W.xxz_chain(6, seed=1)
    for bad in ([1.0, 0.5], [-0.1], [0.5, 3.1]):
        with pytest.raises(ValueError):
            O.evolve(H, v0, 3.0, 1e-8, 10, sample_times=bad)
