"""Pins for the oracle's restarted Krylov evolution (Alg. 1): exact solutions, closed forms,
invariants, forward-backward, resume, Arnoldi relations, the step rule and error paths."""

import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr, sector_evolve, xxz_sectors
from workloads.csr import CSR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _within_bound(res, v_exact, tol):
    err = np.linalg.norm(res.v - v_exact)
    assert err <= res.err_bound * (1 + 1e-3) + 1e-13, (err, res.err_bound)
    assert res.err_bound <= tol * (1 + 1e-12)
    return err


@pytest.mark.parametrize("seed,d,density", [(1, 60, 0.08), (2, 200, 0.03), (3, 400, 0.01)])
@pytest.mark.parametrize("tol,m", [(1e-6, 10), (1e-10, 30)])
def test_dense_exact_random_sparse(seed, d, density, tol, m):
    H = random_hermitian_csr(d, density, seed)
    v0 = W.random_state(np.random.default_rng(seed + 100), d)
    t = 3.0
    res = O.evolve(H, v0, t, tol, m)
    _within_bound(res, dense_evolve(H, v0, t), tol)


@pytest.mark.parametrize("L", [5, 7, 9])
def test_dense_exact_xxz(L):
    H, v0 = W.xxz_chain(L, seed=L)
    res = O.evolve(H, v0, 10.0, 1e-8, 20)
    _within_bound(res, dense_evolve(H, v0, 10.0), 1e-8)


def test_full_size_first_workload_by_sectors():
    # XXZ L=12 (d=4096), t=10, tol=1e-8, m=40: exact answer from the magnetisation blocks.
    wl = W.workload("xxz_L12")
    res = O.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m)
    exact = sector_evolve(wl.H, wl.v0, wl.t, xxz_sectors(12))
    err = _within_bound(res, exact, wl.tol)
    assert err < wl.tol
    # Q5 invariants: norm and energy
    A = wl.H.to_scipy()
    assert abs(np.linalg.norm(res.v) - 1) <= res.err_bound + 1e-12
    e0 = np.vdot(wl.v0, A @ wl.v0).real
    e1 = np.vdot(res.v, A @ res.v).real
    assert abs(e1 - e0) <= 2 * wl.H.norm1() * res.err_bound + 1e-12 * wl.H.norm1()


@pytest.mark.parametrize("n_up,expect_breakdown", [(1, True), (2, False)])
def test_magnon_sectors(n_up, expect_breakdown):
    L = 12
    H, _ = W.xxz_chain(L, seed=2)
    sec = xxz_sectors(L)[n_up]
    v0 = np.zeros(H.dim, dtype=complex)
    v0[sec] = W.random_state(np.random.default_rng(9), sec.size)
    res = O.evolve(H, v0, 20.0, 1e-8, 40)
    _within_bound(res, sector_evolve(H, v0, 20.0, [sec]), 1e-8)
    if expect_breakdown:
        assert res.breakdown_dim == sec.size == 12 and res.steps == 1
    else:
        assert res.breakdown_dim == 0 and res.steps >= 2
    assert np.all(res.v[np.setdiff1d(np.arange(H.dim), sec)] == 0)


def test_multiple_of_identity():
    d, c = 50, 1.7
    H = CSR(d, np.arange(d + 1, dtype=np.int32), np.arange(d, dtype=np.int32), np.full(d, c + 0j))
    v0 = W.random_state(np.random.default_rng(1), d)
    res = O.evolve(H, v0, 2.5, 1e-9, 10)
    assert res.breakdown_dim == 1 and res.steps == 1 and res.matvecs == 1
    assert np.allclose(res.v, np.exp(-1j * c * 2.5) * v0, atol=1e-14)
    assert res.err_bound <= 1e-9


def test_diagonal_hamiltonian_phases():
    d = 30
    diag = np.linspace(-2, 2, d)
    H = CSR(d, np.arange(d + 1, dtype=np.int32), np.arange(d, dtype=np.int32), diag + 0j)
    v0 = W.random_state(np.random.default_rng(2), d)
    res = O.evolve(H, v0, 4.0, 1e-9, 8)
    _within_bound(res, np.exp(-1j * diag * 4.0) * v0, 1e-9)


def test_forward_backward_xxz():
    H, v0 = W.xxz_chain(10, seed=5)
    r1 = O.evolve(H, v0, 10.0, 1e-8, 30)
    r2 = O.evolve(H.negated(), r1.v, 10.0, 1e-8, 30)
    assert np.linalg.norm(r2.v - v0) <= (r1.err_bound + r2.err_bound) * (1 + 1e-3) + 1e-12


def test_forward_backward_paper_example():
    """The paper's check on its own model: back at the start within the requested 2 err_max."""
    gold = json.load(open(GOLDEN))["forward_backward"]
    H, v0, _ = W.memory_burden_model()
    r1 = O.evolve(H, v0, gold["t"], gold["err_max"], 40)
    r2 = O.evolve(H.negated(), r1.v, gold["t"], gold["err_max"], 40)
    back = np.linalg.norm(r2.v - v0)
    assert back <= r1.err_bound + r2.err_bound <= gold["printed_requested_bound"]
    # same order of magnitude as the paper's 9.82e-9 (the paper does not state m)
    assert gold["printed_return_error"] / 10 <= back <= gold["printed_requested_bound"]
    # and the forward state is within its own bound of the exact one
    _within_bound(r1, dense_evolve(H, v0, gold["t"]), gold["err_max"])


def test_resume_is_additive():
    H, v0 = W.xxz_chain(9, seed=6)
    full = O.evolve(H, v0, 8.0, 1e-9, 25)
    a = O.evolve(H, v0, 3.0, 1e-9, 25)
    b = O.evolve(H, a.v, 5.0, 1e-9, 25)
    assert np.linalg.norm(b.v - full.v) <= (a.err_bound + b.err_bound + full.err_bound) * (1 + 1e-3) + 1e-12


def test_arnoldi_relations():
    H, v0 = W.xxz_chain(10, seed=8)
    ar = O.arnoldi(H, v0, 30, 1e-12)
    V, M, k = ar.V, ar.M, ar.k
    assert not ar.breakdown and k == 30
    assert np.abs(V.conj().T @ V - np.eye(k)).max() <= 1e-12
    R = -1j * (H.to_scipy() @ V) - V @ M          # = h v_{k+1} e_k^T
    eps_scale = 10 * k * np.finfo(float).eps * H.norm1()
    assert np.linalg.norm(R[:, :-1]) <= eps_scale
    assert abs(np.linalg.norm(R[:, -1]) - ar.h) <= eps_scale
    assert np.abs(M + M.conj().T).max() <= 1e-15          # anti-Hermitian
    assert np.count_nonzero(np.triu(M, 2)) == 0 and np.count_nonzero(np.tril(M, -2)) == 0
    assert np.allclose(M.diagonal().real, 0)


def test_lanczos_form_matches_arnoldi_form():
    # Plain Lanczos on H (real alpha, beta) gives the same |e_k^T exp(M tau) e_1| as Alg. 1's M.
    H, v0 = W.xxz_chain(8, seed=1)
    ar = O.arnoldi(H, v0, 15, 1e-12)
    alpha = (1j * ar.M.diagonal()).real
    beta = ar.M.diagonal(-1).real
    lam1, U1 = O.hessenberg_eig(ar.M)
    lam2, U2 = O.hessenberg_eig(O.hessenberg_from_lanczos(alpha, beta))
    taus = np.linspace(0, 3, 7)
    assert np.allclose(O.bound_integrand(lam1, U1, 1.0)(taus), O.bound_integrand(lam2, U2, 1.0)(taus), atol=1e-14)
    assert np.allclose(np.sort(np.linalg.eigvalsh(np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1))), lam1)


def test_step_rule_invariants():
    wl = W.workload("xxz_L12")
    res = O.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m)
    rate = wl.tol / wl.t
    assert all(s.err <= rate * s.tau for s in res.trace)
    assert abs(sum(s.tau for s in res.trace) - wl.t) <= 1e-12 * wl.t
    assert sum(s.err for s in res.trace) == pytest.approx(res.err_bound, rel=1e-12)
    assert res.t_reached == wl.t and res.matvecs == sum(s.k for s in res.trace)


def test_trivial_and_invalid_inputs():
    H, v0 = W.xxz_chain(5, seed=1)
    r = O.evolve(H, v0, 0.0, 1e-8, 10)
    assert np.array_equal(r.v, v0) and r.steps == 0 and r.err_bound == 0
    r = O.evolve(H, np.zeros(H.dim, complex), 1.0, 1e-8, 10)
    assert not np.any(r.v) and r.steps == 0
    r = O.evolve(H, 3.0 * v0, 2.0, 1e-8, 10)
    r1 = O.evolve(H, v0, 2.0, 1e-8, 10)
    assert np.allclose(r.v, 3.0 * r1.v, atol=1e-14) and r.err_bound == pytest.approx(3 * r1.err_bound)
    for bad in [dict(t=-1.0), dict(t=np.inf), dict(tol=0.0), dict(tol=np.nan), dict(m=1)]:
        args = dict(t=1.0, tol=1e-8, m=10)
        args.update(bad)
        with pytest.raises(ValueError):
            O.evolve(H, v0, args["t"], args["tol"], args["m"])
    bad_v = v0.copy()
    bad_v[0] = np.nan
    with pytest.raises(ValueError):
        O.evolve(H, bad_v, 1.0, 1e-8, 10)


def test_warnings_and_underflow_are_forcible():
    H, v0 = W.xxz_chain(8, seed=2)
    r = O.evolve(H, v0, 1.0, 1e-15, 20)                   # tol below d ||H||_1 eps
    assert r.warnings & O.WARN_NUMERICAL
    r = O.evolve(H, v0, 1.0, 1e-8, 20, O.Options(quad_max_level=1))
    assert r.warnings & O.WARN_QUADRATURE
    with pytest.raises(O.StepUnderflow):
        O.evolve(H, v0, 50.0, 1e-10, 3, O.Options(t_init=50.0, max_halvings=0))


# --- planted mistakes: each must be caught by the dense pin -------------------------------

def _dense_pin_fails(monkeypatch, name, replacement):
    monkeypatch.setattr(O.krylov, name, replacement)
    H = random_hermitian_csr(120, 0.05, 4)
    v0 = W.random_state(np.random.default_rng(4), 120)
    try:
        res = O.krylov.evolve(H, v0, 3.0, 1e-8, 12)
    except Exception:
        return True
    err = np.linalg.norm(res.v - dense_evolve(H, v0, 3.0))
    return err > res.err_bound * (1 + 1e-3) + 1e-13


def test_planted_sign_error_in_phase_is_caught(monkeypatch):
    good = O.krylov.krylov_coefficients
    assert _dense_pin_fails(monkeypatch, "krylov_coefficients", lambda lam, U, tau: good(-lam, U, tau))


def test_planted_transpose_is_caught(monkeypatch):
    good = O.krylov.hessenberg_eig
    assert _dense_pin_fails(monkeypatch, "hessenberg_eig", lambda M: good(M.T))


def test_planted_wrong_residual_norm_is_caught(monkeypatch):
    good = O.krylov.bound_integrand
    assert _dense_pin_fails(monkeypatch, "bound_integrand", lambda lam, U, h: good(lam, U, 1e-3 * h))


def test_planted_superdiagonal_sign_is_caught(monkeypatch):
    good = O.krylov.arnoldi

    def wrong(H, u, m, tol_rate, three_term=False):
        ar = good(H, u, m, tol_rate, three_term)
        M = ar.M.copy()
        k = M.shape[0]
        M[np.arange(k - 1), np.arange(1, k)] *= -1.0      # M_{j,j+1} = +no instead of -no
        return O.ArnoldiResult(ar.V, M, ar.h, ar.k, ar.breakdown)

    assert _dense_pin_fails(monkeypatch, "arnoldi", wrong)


def test_planted_missing_diagonal_is_caught(monkeypatch):
    good = O.krylov.arnoldi

    def wrong(H, u, m, tol_rate, three_term=False):
        ar = good(H, u, m, tol_rate, three_term)
        M = ar.M - np.diag(ar.M.diagonal())               # dropped M_jj term
        return O.ArnoldiResult(ar.V, M, ar.h, ar.k, ar.breakdown)

    assert _dense_pin_fails(monkeypatch, "arnoldi", wrong)
