"""Pins for the oracle's three-term mode (step 1 with the recurrence exactly as printed in
eq. arnoldi / Alg. 1, no re-orthogonalisation): the bound of eq. errorIntegral still holds
against exact answers, the Arnoldi relation holds to rounding while orthogonality is lost,
short bases agree with the full mode, and a planted sign error in the recurrence is caught."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr, sector_evolve, xxz_sectors


def _within_bound(res, v_exact, tol):
    err = np.linalg.norm(res.v - v_exact)
    assert err <= res.err_bound * (1 + 1e-3) + 1e-13, (err, res.err_bound)
    assert res.err_bound <= tol * (1 + 1e-12)
    return err


@pytest.mark.parametrize("seed,d,density", [(1, 60, 0.08), (2, 200, 0.03), (3, 400, 0.01)])
@pytest.mark.parametrize("tol,m", [(1e-6, 10), (1e-10, 30), (1e-8, 60)])
def test_dense_exact_random_sparse(seed, d, density, tol, m):
    H = random_hermitian_csr(d, density, seed)
    v0 = W.random_state(np.random.default_rng(seed + 100), d)
    res = O.evolve(H, v0, 3.0, tol, m, three_term=True)
    _within_bound(res, dense_evolve(H, v0, 3.0), tol)


@pytest.mark.parametrize("L,m", [(7, 20), (9, 40), (10, 64)])
def test_dense_exact_xxz(L, m):
    H, v0 = W.xxz_chain(L, seed=L)
    res = O.evolve(H, v0, 10.0, 1e-8, m, three_term=True)
    _within_bound(res, dense_evolve(H, v0, 10.0), 1e-8)


def test_first_workload_by_sectors():
    wl = W.workload("xxz_L12")
    res = O.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, three_term=True)
    _within_bound(res, sector_evolve(wl.H, wl.v0, wl.t, xxz_sectors(12)), wl.tol)


def test_relation_holds_while_orthogonality_is_lost():
    H, v0 = W.xxz_chain(10, seed=8)
    full = O.arnoldi(H, v0, 60, 1e-12)
    three = O.arnoldi(H, v0, 60, 1e-12, three_term=True)
    assert full.k == three.k == 60
    orth = lambda V: np.abs(V.conj().T @ V - np.eye(V.shape[1])).max()
    # no full pass: orthogonality decays by orders of magnitude (the full mode keeps ~1e-15)
    assert orth(full.V) <= 1e-13
    assert orth(three.V) >= 1e-8
    # the Arnoldi relation A V - V M = h v_{k+1} e_k^T still holds to rounding, and M is the
    # anti-Hermitian tridiagonal of Alg. 1
    V, M = three.V, three.M
    R = -1j * (H.to_scipy() @ V) - V @ M
    eps_scale = 10 * 60 * np.finfo(float).eps * H.norm1()
    assert np.linalg.norm(R[:, :-1]) <= eps_scale
    assert abs(np.linalg.norm(R[:, -1]) - three.h) <= eps_scale
    assert np.abs(M + M.conj().T).max() <= 1e-15
    assert np.count_nonzero(np.triu(M, 2)) == 0 and np.count_nonzero(np.tril(M, -2)) == 0
    # columns stay unit vectors (each one is normalised by its computed residual norm)
    assert np.abs(np.linalg.norm(V, axis=0) - 1).max() <= 1e-14


def test_short_bases_agree_with_full_mode():
    H, v0 = W.xxz_chain(9, seed=4)
    a = O.arnoldi(H, v0, 8, 1e-12)
    b = O.arnoldi(H, v0, 8, 1e-12, three_term=True)
    assert np.abs(a.M - b.M).max() <= 1e-12 * H.norm1()
    assert np.abs(a.V - b.V).max() <= 1e-12
    ra = O.evolve(H, v0, 2.0, 1e-8, 8)
    rb = O.evolve(H, v0, 2.0, 1e-8, 8, three_term=True)
    assert ra.steps == rb.steps
    assert np.linalg.norm(ra.v - rb.v) <= 1e-11


def test_planted_recurrence_sign_is_caught(monkeypatch):
    # subtracting +beta v_{j-1} where Alg. 1 subtracts M_{j-1,j} v_{j-1} = -beta v_{j-1}
    def wrong(H, u, m, tol_rate, three_term=False):
        mat = H.to_scipy()
        d = u.shape[0]
        V = np.zeros((d, m), dtype=np.complex128)
        M = np.zeros((m, m), dtype=np.complex128)
        V[:, 0] = u
        h = 0.0
        for j in range(m):
            p = -1j * (mat @ V[:, j])
            if j > 0:
                p = p + M[j - 1, j] * V[:, j - 1]
            M[j, j] = np.vdot(V[:, j], p)
            p = p - M[j, j] * V[:, j]
            no = float(np.linalg.norm(p))
            if j < m - 1:
                M[j, j + 1] = -no
                M[j + 1, j] = no
                V[:, j + 1] = p / no
            else:
                h = no
        return O.ArnoldiResult(V, M, h, m, False)

    monkeypatch.setattr(O.krylov, "arnoldi", wrong)
    H = random_hermitian_csr(120, 0.05, 4)
    v0 = W.random_state(np.random.default_rng(4), 120)
    failed = False
    try:
        res = O.krylov.evolve(H, v0, 3.0, 1e-8, 12, three_term=True)
        failed = np.linalg.norm(res.v - dense_evolve(H, v0, 3.0)) > res.err_bound * (1 + 1e-3) + 1e-13
    except Exception:
        failed = True
    assert failed
