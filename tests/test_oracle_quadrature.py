"""Pins for the oracle's tanh-sinh rule: closed forms, an arbitrary-precision reference,
the node layout, and the non-convergence flag."""

import math

import mpmath
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.quadrature import level_nodes


def test_node_layout():
    for level in range(6):
        total = sum(level_nodes(l).size for l in range(level + 1))
        assert total == 6 * 2 ** level + 1
    all_u = np.sort(np.concatenate([level_nodes(l) for l in range(4)]))
    assert np.allclose(np.diff(all_u), 2.0 ** -3) and all_u[0] == -3 and all_u[-1] == 3


@pytest.mark.parametrize("a,b", [(0.0, 1.0), (0.3, 7.5), (2.0, 2.5)])
def test_constant_and_polynomial(a, b):
    r = O.tanh_sinh(lambda x: np.ones_like(x), a, b)
    assert r.converged and abs(r.value - (b - a)) <= 1e-12 * (b - a)
    r = O.tanh_sinh(lambda x: x ** 3, a, b)
    assert abs(r.value - (b ** 4 - a ** 4) / 4) <= 1e-6 * (b ** 4 - a ** 4) / 4


def test_two_level_closed_form():
    # 2x2 block J = [[a1, beta], [beta, a2]]: |e_2^T exp(-iJt) e_1| = (2 beta/dl) |sin(dl t/2)|,
    # dl = sqrt((a1-a2)^2 + 4 beta^2); its integral up to 2 pi / dl is (4 beta / dl^2)(1 - cos(dl t/2)).
    a1, a2, beta, h = 0.3, -1.1, 0.7, 0.9
    dl = math.sqrt((a1 - a2) ** 2 + 4 * beta ** 2)
    M = O.hessenberg_from_lanczos(np.array([a1, a2]), np.array([beta]))
    lam, U = O.hessenberg_eig(M)
    f = O.bound_integrand(lam, U, h)
    taus = np.linspace(0, 2 * math.pi / dl, 9)
    assert np.allclose(f(taus), h * (2 * beta / dl) * np.abs(np.sin(dl * taus / 2)), atol=1e-14)
    for tau in taus[1:]:
        exact = h * (4 * beta / dl ** 2) * (1 - math.cos(dl * tau / 2))
        r = O.tanh_sinh(f, 0.0, tau)
        assert r.converged and abs(r.value - exact) <= 1e-3 * exact


def test_small_tau_power_law():
    # For a k x k unreduced tridiagonal, e_k^T exp(-iJ tau) e_1 = (-i tau)^(k-1) prod(beta)/(k-1)! + O(tau^k)
    rng = np.random.default_rng(5)
    k = 4
    alpha, beta = rng.uniform(-1, 1, k), rng.uniform(0.5, 1.5, k - 1)
    lam, U = O.hessenberg_eig(O.hessenberg_from_lanczos(alpha, beta))
    h = 0.8
    f = O.bound_integrand(lam, U, h)
    tau = 1e-3
    lead = h * np.prod(beta) * tau ** k / math.factorial(k)
    r = O.tanh_sinh(f, 0.0, tau)
    assert abs(r.value - lead) <= 1e-2 * lead


def test_against_mpmath_on_captured_integrands():
    H, v0 = W.xxz_chain(8, seed=4)
    ar = O.arnoldi(H, v0, 12, 1e-12)
    lam, U = O.hessenberg_eig(ar.M)
    f = O.bound_integrand(lam, U, ar.h)
    k = lam.size
    coef = [mpmath.mpc(complex(z)) for z in U[k - 1, :] * np.conj(U[0, :])]
    lam_mp = [mpmath.mpf(float(x)) for x in lam]

    def f_mp(tau):
        return ar.h * abs(sum(c * mpmath.exp(-1j * l * tau) for c, l in zip(coef, lam_mp)))

    mpmath.mp.dps = 30
    for a, b in [(0.0, 0.5), (0.0, 2.0), (1.0, 1.3), (0.0, 6.0)]:
        ref = float(mpmath.quad(f_mp, [a, b], method="tanh-sinh"))
        r = O.tanh_sinh(f, a, b)
        assert r.converged and abs(r.value - ref) <= 1e-3 * ref, (a, b, r.value, ref)


def test_nonconvergence_is_flagged():
    r = O.tanh_sinh(lambda x: np.abs(np.sin(400 * x)), 0.0, 10.0, max_level=2)
    assert not r.converged
    r = O.tanh_sinh(lambda x: np.ones_like(x), 0.0, 1.0, max_level=1)  # min_level 3 unreachable
    assert not r.converged


def test_noise_floor_accepts_zero_and_tiny():
    r = O.tanh_sinh(lambda x: np.zeros_like(x), 0.0, 1.0)
    assert r.converged and r.value == 0.0 and r.level == 3
    rng = np.random.default_rng(0)
    noise = lambda x: 1e-17 * rng.random(x.shape)
    assert not O.tanh_sinh(noise, 0.0, 1.0, max_level=8).converged
    assert O.tanh_sinh(noise, 0.0, 1.0, max_level=8, abs_tol=1e-16).converged
