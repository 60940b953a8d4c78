"""Pins for the step search of Alg. 1 step 2 (eq. stepSize), in particular its substep loop.

The printed substep loop integrates over intervals whose bounds are garbled; the reading
adopted (R4) integrates [tau + (n-1) s, tau + n s] for the n-th substep, so that the error
attached to the returned step is the integral of eq. errorIntegral over [0, tau] exactly.
Every pin below checks that identity against a value computed without the oracle's
quadrature: closed-form integrals of integrands driven through ``step_size`` on the first-step
and later-step paths, an integrand whose only feature lies inside the first substep interval,
and every accepted step of real evolutions against QUADPACK (adaptive Gauss-Kronrod, a
different method from the oracle's tanh-sinh rule).  A planted shift of the substep intervals
by one substep (the literal reading, which skips [tau, tau + s]) must fail each pin."""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
import workloads as W
from tests.exact import random_hermitian_csr

EPS = 2.0 ** -52


def _poly_pin(first: bool, tau_prev: float, expect_tau: float) -> bool:
    """f(x) = c x^2 with c = 2.9 and rate 1: the rate holds exactly for tau < sqrt(3 / 2.9)."""
    c, rate, t_rem = 2.9, 1.0, 10.0
    tau, err, ok = O.step_size(lambda x: c * np.asarray(x) ** 2, rate, t_rem, first, tau_prev, False)
    assert ok
    assert tau == pytest.approx(expect_tau, rel=1e-12)
    return abs(err - c * tau ** 3 / 3) <= 1e-9 * c * tau ** 3 / 3


def test_substeps_first_path_closed_form():
    # doubling 0.1 -> 0.8 (1.6 breaks the rate), then substeps of 0.08 up to 0.96 (1.04 breaks it)
    assert _poly_pin(True, 0.1, 0.96)


def test_substeps_later_path_closed_form():
    # 0.97 * tau_prev = 0.5: ten substeps of 0.05 accepted, up to 1.0 (1.05 breaks the rate)
    assert _poly_pin(False, 0.5 / 0.97, 1.0)
    # 0.97 * tau_prev = 3: halved twice to 0.75, then substeps of 0.075 up to 0.975
    assert _poly_pin(False, 3.0 / 0.97, 0.975)


def _two_level_pin(first: bool, tau_prev: float) -> bool:
    # 2x2 block: f = h (2 beta / dl) |sin(dl x / 2)|, integral h (4 beta / dl^2)(1 - cos(dl x / 2))
    # for dl x <= 2 pi.
    a1, a2, beta, h = 0.3, -1.1, 0.7, 0.9
    dl = math.sqrt((a1 - a2) ** 2 + 4 * beta ** 2)
    lam, U = O.hessenberg_eig(O.hessenberg_from_lanczos(np.array([a1, a2]), np.array([beta])))
    f = O.bound_integrand(lam, U, h)
    tau, err, ok = O.step_size(f, 0.35, 50.0, first, tau_prev, False)
    assert ok and dl * tau <= 2 * math.pi
    exact = h * (4 * beta / dl ** 2) * (1 - math.cos(dl * tau / 2))
    return abs(err - exact) <= 1e-9 * exact


@pytest.mark.parametrize("first,tau_prev", [(True, 0.1), (False, 1.0), (False, 2.3)])
def test_substeps_two_level_closed_form(first, tau_prev):
    assert _two_level_pin(first, tau_prev)


def _bump_integrand():
    """A floor, a C^1 bump of area A on [1.02, 1.07] and a cubic-growing part: the later-step
    path starts at tau = 1.0 with substeps of 0.1, so the bump lies inside the first substep
    interval only."""
    eps0, A, a, w, c = 1e-3, 0.02, 1.02, 0.05, 0.03

    def f(x):
        x = np.asarray(x, dtype=np.float64)
        inside = (x >= a) & (x <= a + w)
        bump = np.where(inside, A * (1 - np.cos(2 * np.pi * (x - a) / w)) / w, 0.0)
        return eps0 + bump + c * x ** 2

    def integral(x):
        return eps0 * x + (A if x >= a + w else 0.0) + c * x ** 3 / 3

    return f, integral


def _bump_pin() -> bool:
    f, integral = _bump_integrand()
    tau, err, _ = O.step_size(f, 0.05, 100.0, False, 1.0 / 0.97, False)
    assert tau == pytest.approx(1.9, rel=1e-12)       # substeps 1.1 .. 1.9 accepted, 2.0 is not
    exact = integral(tau)
    return abs(err - exact) <= 1e-3 * exact


def test_substep_covers_first_interval():
    assert _bump_pin()


def _capture_runs(monkeypatch):
    """Evolutions whose integrands are recorded as the oracle builds them (one per restart)."""
    captured = []
    good = O.krylov.bound_integrand

    def recording(lam, U, h):
        captured.append((lam.copy(), U.copy(), float(h)))
        return good(lam, U, h)

    monkeypatch.setattr(O.krylov, "bound_integrand", recording)
    runs = []
    H = random_hermitian_csr(200, 0.03, 2)
    v0 = W.random_state(np.random.default_rng(102), 200)
    for (Hm, v, t, tol, m) in [(H, v0, 3.0, 1e-6, 10), (H, v0, 3.0, 1e-10, 16)] + \
            [(W.xxz_chain(9, seed=9)[0], W.xxz_chain(9, seed=9)[1], 10.0, 1e-8, 20)]:
        captured.clear()
        res = O.krylov.evolve(Hm, v, t, tol, m)
        runs.append((res, list(captured), t))
    monkeypatch.undo()
    return runs


def _substeps_used(trace, t, t_init=0.1, shrink=0.97):
    """Steps whose size is none of the search's candidates (doublings / halvings of the start,
    or the remaining time): those were extended by accepted substeps."""
    used, t_now = 0, 0.0
    for k, s in enumerate(trace):
        t_rem = t - t_now
        start = min(t_init, t_rem) if k == 0 else min(shrink * trace[k - 1].tau, t_rem)
        cands = [start * 2.0 ** e for e in range(-64, 40)] + [t_rem]
        if not any(abs(s.tau - c) <= 1e-14 * c for c in cands):
            used += 1
        t_now += s.tau
    return used


def _captured_pin(runs) -> bool:
    for res, caps, t in runs:
        assert len(caps) == len(res.trace)
        for (lam, U, h), s in zip(caps, res.trace):
            f = O.bound_integrand(lam, U, h)
            floor = h * lam.size * EPS * s.tau           # rounding floor of f times the interval
            ref, _ = integrate.quad(lambda x: float(f(x)[0]), 0.0, s.tau, epsabs=floor, epsrel=1e-10, limit=400)
            if abs(s.err - ref) > 1e-3 * ref + floor:
                return False
    return True


def test_every_accepted_step_matches_an_independent_integral(monkeypatch):
    runs = _capture_runs(monkeypatch)
    assert sum(_substeps_used(res.trace, t) for res, _, t in runs) >= 3
    assert _captured_pin(runs)


# --- planted mistake: the literal substep bounds, shifted one substep to the right ----------

def _plant_shifted_substeps(monkeypatch):
    """Only substep integrals start away from 0; shift each of them by its own width, so the
    n-th substep integrates [tau + n s, tau + (n + 1) s]."""
    good = O.krylov.tanh_sinh

    def shifted(f, a, b, *args, **kw):
        if a > 0.0:
            a, b = b, 2.0 * b - a
        return good(f, a, b, *args, **kw)

    monkeypatch.setattr(O.krylov, "tanh_sinh", shifted)


def test_planted_substep_shift_fails_every_pin(monkeypatch):
    _plant_shifted_substeps(monkeypatch)
    assert not _poly_pin(True, 0.1, 0.96)
    assert not _two_level_pin(True, 0.1)
    f, integral = _bump_integrand()
    tau, err, _ = O.krylov.step_size(f, 0.05, 100.0, False, 1.0 / 0.97, False)
    assert abs(err - integral(tau)) > 1e-3 * integral(tau)
    runs = _capture_runs(monkeypatch)   # undoes the plant after the runs
    assert not _captured_pin(runs)
