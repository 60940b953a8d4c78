"""Pins for the oracle's fast integration option (Sec. "Description of Program": a non-adaptive
Gauss scheme for the error integral): the n-point rule integrates polynomials of degree
2n - 1 exactly and misses degree 2n; on captured bound integrands it agrees with the adaptive
rule; evolutions in this mode stay within tol of exact answers on smooth problems."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr


@pytest.mark.parametrize("n", [1, 2, 5, 16, 40])
def test_polynomial_exactness(n):
    rng = np.random.default_rng(n)
    c = rng.standard_normal(2 * n)            # degree 2n - 1
    a, b = -0.7, 1.9
    f = lambda x: np.polyval(c, x)
    exact = np.polyval(np.polyint(c), b) - np.polyval(np.polyint(c), a)
    got = O.gauss_legendre(f, a, b, n).value
    assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact))
    if n <= 5:  # degree 2n is not integrated exactly: x^(2n) on [-1, 1] has error ~ 4^-n
        g = lambda x: x ** (2 * n)
        exact2 = 2.0 / (2 * n + 1)
        assert abs(O.gauss_legendre(g, -1.0, 1.0, n).value - exact2) > 1e-6 * exact2


def test_agrees_with_adaptive_rule_on_bound_integrands():
    H, v0 = W.xxz_chain(9, seed=2)
    ar = O.arnoldi(H, v0, 20, 1e-12)
    lam, U = O.hessenberg_eig(ar.M)
    f = O.bound_integrand(lam, U, ar.h)
    for tau in (0.05, 0.3, 1.0):
        ref = O.tanh_sinh(f, 0.0, tau, 1e-12, 20, 3, 0.0).value
        got = O.gauss_legendre(f, 0.0, tau, 32).value
        floor = 2 * ar.h * ar.k * np.finfo(float).eps * tau  # rounding floor of the integrand
        assert abs(got - ref) <= 1e-9 * abs(ref) + floor, (tau, got, ref)


@pytest.mark.parametrize("n", [8, 32])
def test_evolution_in_gauss_mode(n):
    H = random_hermitian_csr(200, 0.03, 5)
    v0 = W.random_state(np.random.default_rng(6), 200)
    opts = O.Options(quad_gauss_points=n)
    res = O.evolve(H, v0, 3.0, 1e-8, 20, opts)
    ref = O.evolve(H, v0, 3.0, 1e-8, 20)
    err = np.linalg.norm(res.v - dense_evolve(H, v0, 3.0))
    assert err <= 1e-8
    assert res.warnings & O.WARN_QUADRATURE == 0
    # the fixed rule approximates the same integrals: bounds agree closely
    assert abs(res.err_bound - ref.err_bound) <= 0.05 * ref.err_bound
