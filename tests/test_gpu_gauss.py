"""The fast integration option (te_options.quad_gauss_points = n: the n-point Gauss-Legendre
rule per error integral, Sec. "Description of Program") through the C ABI: the device rule
against numpy's Legendre nodes on bound integrands, and whole evolutions against the oracle in
the same mode (||v_gpu - v_oracle|| <= 2 tol + 1e-12)."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 7, 16, 40, 64])
def test_device_rule_matches_numpy_legendre(n):
    announce(f"gauss rule n={n}")
    te = lib()
    H, v0 = W.xxz_chain(9, seed=4)
    ar = O.arnoldi(H, v0, 24, 1e-12)
    lam, U = O.hessenberg_eig(ar.M)
    k = lam.size
    coef = (U[k - 1, :] * np.conj(U[0, :])).real  # the Lanczos form's coefficients are real
    f = lambda tau: ar.h * np.abs(np.exp(-1j * np.outer(np.atleast_1d(tau), lam)) @ coef)
    for a, b in [(0.0, 0.4), (0.3, 1.7)]:
        got, level, conv = te.te_error_integral(lam, coef, ar.h, a, b, options=te.te_default_options(quad_gauss_points=n))
        want = O.gauss_legendre(f, a, b, n).value
        floor = 4 * ar.h * k * np.finfo(float).eps * (b - a)
        assert abs(got - want) <= 1e-12 * abs(want) + floor, (n, a, b, got, want)
        assert conv


@pytest.mark.parametrize("n", [16, 32])
def test_evolution_in_gauss_mode_matches_oracle(n):
    announce(f"gauss evolve n={n}")
    te = lib()
    wl = W.workload("xxz_L12")
    with hamiltonian(wl.H) as h:
        v, res = te.te_evolve(h, to_dev(wl.v0), wl.t, wl.tol, wl.m, options=te.te_default_options(quad_gauss_points=n))
        v = to_host(v)
    ro = O.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, O.Options(quad_gauss_points=n))
    assert np.linalg.norm(v - ro.v) <= 2 * wl.tol + 1e-12
    assert not (res.warnings & te.TE_WARN_QUADRATURE)
    assert abs(res.err_bound - ro.err_bound) <= 0.05 * ro.err_bound


def test_gauss_mode_on_random_hermitian():
    announce("gauss random")
    te = lib()
    H = random_hermitian_csr(500, 0.02, 9)
    v0 = W.random_state(np.random.default_rng(10), 500)
    with hamiltonian(H) as h:
        v, res = te.te_evolve(h, to_dev(v0), 3.0, 1e-9, 24, options=te.te_default_options(quad_gauss_points=24))
    assert np.linalg.norm(to_host(v) - dense_evolve(H, v0, 3.0)) <= 1e-9
    with pytest.raises(te.TEError):
        with hamiltonian(H) as h2:
            te.te_evolve(h2, to_dev(v0), 3.0, 1e-9, 24, options=te.te_default_options(quad_gauss_points=65))
