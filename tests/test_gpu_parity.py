"""Parity of the HIP path (called through the C ABI) with the CPU oracle, step by step and end
to end, plus the ABI's error paths.  Tolerances:
  sparse product          relative 1e-13 (FP64, <= 23 terms per row)
  alpha / beta            1e-11 relative to ||H||_1 (different orthogonalisation order)
  basis orthogonality     1e-12
  eigen-decomposition     residual 50 k eps ||J||, orthogonality 50 k eps
  quadrature              1e-12 relative to the oracle on identical inputs (same nodes), or
                          2 h k eps (b - a): f = h|sum_n c_n exp(-i lam_n tau)| is known only to
                          within its rounding floor h k eps, so integrals at that floor differ
                          between any two FP64 evaluations
  evolution               ||v_gpu - v_oracle|| <= 2 tol + 1e-12 and each within its bound
                          of the exact answer where one is available."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr, sector_evolve, xxz_sectors
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


# ------------------------------------------------------------------ a1: sparse product
@pytest.mark.parametrize("case", ["xxz8", "rand1000", "rand1537", "bose6", "xxz20"])
def test_spmv_matches_scipy(case):
    announce(f"spmv {case}")
    if case == "xxz8":
        H, x = W.xxz_chain(8, seed=1)
    elif case == "xxz20":
        H, x = W.xxz_chain(20, seed=2)
    elif case == "bose6":
        H, x = W.bosonic_chain(6, 6, seed=3)
    else:
        d = int(case[4:])
        H = random_hermitian_csr(d, 0.01, seed=d)
        x = W.random_state(np.random.default_rng(d), d)
    te = lib()
    with hamiltonian(H) as h:
        y, xhy = te.te_spmv(h, to_dev(x))
        y = to_host(y)
    ref = H.to_scipy() @ x
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    assert abs(xhy - np.vdot(x, ref)) <= 1e-12 * np.linalg.norm(ref)
    assert h.norm1 == pytest.approx(H.norm1(), rel=1e-13)


# ------------------------------------------------------- a2/a3: Krylov build (Lanczos form)
@pytest.mark.parametrize("L,m", [(8, 20), (10, 40), (12, 64)])
def test_arnoldi_matches_oracle(L, m):
    announce(f"arnoldi L={L} m={m}")
    H, u = W.xxz_chain(L, seed=L + 1)
    te = lib()
    with hamiltonian(H) as h:
        V, alpha, beta, k = te.te_arnoldi(h, to_dev(u), m, 1e-12)
        V = to_host(V)
    ar = O.arnoldi(H, u, m, 1e-12)
    assert k == ar.k
    a_ref = (1j * ar.M.diagonal()).real
    b_ref = np.append(ar.M.diagonal(-1).real, ar.h)
    scale = H.norm1()
    assert np.abs(alpha - a_ref).max() <= 1e-11 * scale
    assert np.abs(beta - b_ref).max() <= 1e-11 * scale
    G = V.conj() @ V.T
    assert np.abs(G - np.eye(k)).max() <= 1e-12
    # Lanczos relation H V^T = V^T J + beta_k v_{k+1} e_k^T: the first k-1 columns vanish
    A = H.to_scipy()
    J = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    R = A @ V.T - V.T @ J
    assert np.linalg.norm(R[:, :-1]) <= 10 * k * EPS * scale
    assert abs(np.linalg.norm(R[:, -1]) - beta[-1]) <= 10 * k * EPS * scale


def test_arnoldi_breakdown_in_small_sector():
    announce("arnoldi breakdown")
    L = 10
    H, _ = W.xxz_chain(L, seed=4)
    sec = xxz_sectors(L)[1]
    u = np.zeros(H.dim, complex)
    u[sec] = W.random_state(np.random.default_rng(1), sec.size)
    te = lib()
    with hamiltonian(H) as h:
        V, alpha, beta, k = te.te_arnoldi(h, to_dev(u), 40, 1e-10)
    ar = O.arnoldi(H, u, 40, 1e-10)
    assert ar.breakdown and k == ar.k == L
    assert beta[-1] < 1e-10


def test_arnoldi_full_size_first_steps():
    announce("arnoldi L=20 m=8")
    wl = W.workload("xxz_L20")
    te = lib()
    with hamiltonian(wl.H) as h:
        V, alpha, beta, k = te.te_arnoldi(h, to_dev(wl.v0), 8, 1e-12)
    ar = O.arnoldi(wl.H, wl.v0, 8, 1e-12)
    assert np.abs(alpha - (1j * ar.M.diagonal()).real).max() <= 1e-11 * wl.H.norm1()
    assert np.abs(beta[:-1] - ar.M.diagonal(-1).real).max() <= 1e-11 * wl.H.norm1()


# ------------------------------------------------------------ a4: tridiagonal eigensolver
def _tridiag_cases():
    rng = np.random.default_rng(7)
    cases = {}
    for k in (1, 2, 3, 7, 40, 60, 64):
        cases[f"rand{k}"] = (rng.uniform(-3, 3, k), rng.uniform(0.1, 2, max(k - 1, 0)))
    k = 21  # Wilkinson W21+: pairs of nearly equal eigenvalues
    cases["wilkinson21"] = (np.abs(np.arange(k) - 10.0), np.ones(k - 1))
    cases["tiny_beta"] = (rng.uniform(-1, 1, 30), np.full(29, 1e-9))
    cases["graded"] = (np.logspace(-8, 2, 40), np.logspace(-6, 1, 39))
    cases["constant"] = (np.full(16, 0.5), np.full(15, 1.0))
    # divide and conquer (k >= 16) splits at k // 2: coupling there exactly zero, tiny, negative;
    # identical halves (pairs of equal poles: rotation deflation); sizes around the switch
    b = rng.uniform(0.1, 2, 39)
    b[19] = 0.0
    cases["split_zero"] = (rng.uniform(-3, 3, 40), b)
    b = rng.uniform(0.1, 2, 39)
    b[19] = 1e-300
    cases["split_tiny"] = (rng.uniform(-3, 3, 40), b)
    cases["negative_beta"] = (rng.uniform(-3, 3, 40), -rng.uniform(0.1, 2, 39))
    h, e = rng.uniform(-3, 3, 20), rng.uniform(0.1, 2, 19)
    cases["equal_halves"] = (np.r_[h, h], np.r_[e, 1e-3, e])
    cases["zero_diagonal"] = (np.zeros(40), np.ones(39))
    cases["wide_range"] = (rng.uniform(-1e6, 1e6, 40), rng.uniform(1e-3, 1.0, 39))
    for k in (15, 17, 63):
        cases[f"rand{k}"] = (rng.uniform(-3, 3, k), rng.uniform(0.1, 2, k - 1))
    H, v0 = W.xxz_chain(12, seed=2)
    ar = O.arnoldi(H, v0, 40, 1e-300)
    cases["lanczos_xxz12"] = ((1j * ar.M.diagonal()).real, ar.M.diagonal(-1).real)
    return cases


@pytest.mark.parametrize("name", list(_tridiag_cases()))
def test_tridiag_eig(name):
    announce(f"eig {name}")
    a, b = _tridiag_cases()[name]
    k = a.size
    lam, Q = lib().te_tridiag_eig(a, b)
    J = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    nJ = np.abs(J).sum(axis=0).max()
    assert np.linalg.norm(J @ Q - Q * lam) <= 50 * k * EPS * nJ
    assert np.abs(Q.T @ Q - np.eye(k)).max() <= 50 * k * EPS
    assert np.abs(np.sort(lam) - np.linalg.eigvalsh(J)).max() <= 50 * k * EPS * nJ


# --------------------------------------------------------------- a5: error integral + step
def _spectrum(k, seed):
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-2, 2, k), rng.uniform(0.3, 1.5, k - 1)
    lam, U = O.hessenberg_eig(O.hessenberg_from_lanczos(a, b))
    return a, b, lam, U


@pytest.mark.parametrize("k,a,bnd", [(2, 0.0, 1.0), (6, 0.0, 0.3), (12, 0.5, 2.5), (40, 0.0, 4.0), (40, 1.0, 1.1),
                                     (40, 5.0, 30.0), (64, 0.0, 50.0), (20, 0.0, 12.0)])
def test_error_integral_matches_oracle(k, a, bnd):
    announce(f"integral k={k} [{a},{bnd}]")
    al, be, lam, U = _spectrum(k, k)
    h = 0.7
    # device input: real eigenvectors of J (same eigenvalues as Alg. 1's iM)
    J = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    lam_j, Q = np.linalg.eigh(J)
    val, level, conv = lib().te_error_integral(lam_j, Q[k - 1, :] * Q[0, :], h, a, bnd)
    f = O.bound_integrand(lam, U, h)
    floor = h * k * 2.0 ** -52 * (bnd - a)
    ref = O.tanh_sinh(f, a, bnd, abs_tol=floor)
    assert conv == ref.converged
    assert abs(val - ref.value) <= 1e-12 * abs(ref.value) + 2 * floor
    if ref.value > 1e3 * floor:  # well above the floor both sides take the same number of levels
        assert level == ref.level


@pytest.mark.parametrize("k,first,breakdown,tau_prev,t_rem", [
    (10, True, False, 0.1, 100.0), (20, False, False, 1.3, 50.0), (40, True, False, 0.1, 10.0),
    (40, False, False, 4.0, 3.0), (5, False, True, 1.0, 7.0), (30, False, False, 0.05, 0.07)])
def test_step_search_matches_oracle(k, first, breakdown, tau_prev, t_rem):
    announce(f"step k={k} first={first} bd={breakdown}")
    a, b, lam, U = _spectrum(k, 100 + k)
    h = 1e-10 if breakdown else 0.4
    rate = 1e-10
    tau, err, omega, warn = lib().te_step_search(a, b, h, rate, t_rem, first, tau_prev, breakdown)
    f = O.bound_integrand(lam, U, h)
    tau_o, err_o, ok = O.step_size(f, rate, t_rem, first, tau_prev, breakdown, noise_rate=h * k * 2.0 ** -52)
    assert tau == pytest.approx(tau_o, rel=1e-12)
    assert abs(err - err_o) <= 1e-9 * abs(err_o) + 2 * h * k * 2.0 ** -52 * tau
    assert err <= rate * tau * (1 + 1e-12)
    # omega in the Lanczos basis = D^H (omega of Alg. 1 in the A = -iH basis), D = diag((-i)^j)
    om_o = O.krylov_coefficients(lam, U, tau) * (-1j) ** np.arange(k)
    assert np.abs(omega - om_o).max() <= 1e-12
    assert warn == (0 if ok else 2)


# --------------------------------------------------------------- a1-a7: whole evolution
def _evolve_gpu(H, v0, t, tol, m, **opts):
    te = lib()
    options = te.te_default_options(**opts) if opts else None
    with hamiltonian(H) as h:
        v, res = te.te_evolve(h, to_dev(v0), t, tol, m, options=options)
        return to_host(v), res


def _assert_parity(H, v0, t, tol, m, exact=None):
    v, res = _evolve_gpu(H, v0, t, tol, m)
    ro = O.evolve(H, v0, t, tol, m)
    assert res.t_reached == t
    assert np.linalg.norm(v - ro.v) <= 2 * tol + 1e-12
    assert res.err_bound <= tol * (1 + 1e-12)
    assert abs(res.steps - ro.steps) <= 1
    assert res.err_bound == pytest.approx(ro.err_bound, rel=0.05) or abs(res.steps - ro.steps) == 1
    if exact is not None:
        assert np.linalg.norm(v - exact) <= res.err_bound * (1 + 1e-3) + 1e-12
    return v, res, ro


def test_evolve_first_workload_parity():
    announce("evolve xxz_L12")
    wl = W.workload("xxz_L12")
    exact = sector_evolve(wl.H, wl.v0, wl.t, xxz_sectors(12))
    v, res, ro = _assert_parity(wl.H, wl.v0, wl.t, wl.tol, wl.m, exact)
    assert res.steps == ro.steps and res.matvecs == ro.matvecs
    A = wl.H.to_scipy()
    assert abs(np.linalg.norm(v) - 1) <= res.err_bound + 1e-12
    assert abs(np.vdot(v, A @ v).real - np.vdot(wl.v0, A @ wl.v0).real) <= 2 * wl.H.norm1() * res.err_bound + 1e-11


@pytest.mark.parametrize("d,seed,m,tol", [(300, 1, 10, 1e-6), (1000, 2, 30, 1e-10), (1537, 3, 64, 1e-8),
                                          (70, 4, 64, 1e-8)])
def test_evolve_random_sparse_parity(d, seed, m, tol):
    announce(f"evolve random d={d} m={m}")
    H = random_hermitian_csr(d, min(0.05, 8.0 / d), seed)
    v0 = W.random_state(np.random.default_rng(seed), d)
    _assert_parity(H, v0, 4.0, tol, m, dense_evolve(H, v0, 4.0))


def test_evolve_bosonic_and_paper_model():
    announce("evolve bose K6 / memory-burden")
    H, v0 = W.bosonic_chain(6, 6, seed=3)
    _assert_parity(H, v0, 5.0, 1e-10, 30, dense_evolve(H, v0, 5.0))
    H, v0, _ = W.memory_burden_model()
    v1, r1, _ = _assert_parity(H, v0, 10.0, 1e-8, 40, dense_evolve(H, v0, 10.0))
    v2, r2 = _evolve_gpu(H.negated(), v1, 10.0, 1e-8, 40)
    assert np.linalg.norm(v2 - v0) <= r1.err_bound + r2.err_bound <= 2.0e-8  # paper's forward-backward check


def test_evolve_full_size_sector_pin():
    """XXZ L=20 (full 2^20-row product) with v0 in the 2-magnon sector: exact by a 190x190 eigh."""
    announce("evolve L=20 sector pin")
    L = 20
    H, _ = W.xxz_chain(L, seed=2)
    sec = xxz_sectors(L)[2]
    v0 = np.zeros(H.dim, complex)
    v0[sec] = W.random_state(np.random.default_rng(5), sec.size)
    v, res = _evolve_gpu(H, v0, 30.0, 1e-8, 40)
    exact = sector_evolve(H, v0, 30.0, [sec])
    assert np.linalg.norm(v - exact) <= res.err_bound * (1 + 1e-3) + 1e-12
    assert res.err_bound <= 1e-8 and res.steps >= 2


def test_evolve_full_size_invariants():
    """The benchmarked configuration: XXZ L=20, t=100, tol=1e-8, m=40."""
    announce("evolve xxz_L20 full")
    wl = W.workload("xxz_L20")
    v, res = _evolve_gpu(wl.H, wl.v0, wl.t, wl.tol, wl.m)
    A = wl.H.to_scipy()
    assert res.t_reached == wl.t and res.err_bound <= wl.tol
    assert abs(np.linalg.norm(v) - 1) <= res.err_bound + 1e-12
    e0 = np.vdot(wl.v0, A @ wl.v0).real
    assert abs(np.vdot(v, A @ v).real - e0) <= 2 * wl.H.norm1() * res.err_bound + 1e-11
    assert res.matvecs == 40 * res.steps


def test_evolve_breakdown_lucky():
    announce("evolve breakdown")
    L = 12
    H, _ = W.xxz_chain(L, seed=2)
    sec = xxz_sectors(L)[1]
    v0 = np.zeros(H.dim, complex)
    v0[sec] = W.random_state(np.random.default_rng(9), sec.size)
    v, res = _evolve_gpu(H, v0, 20.0, 1e-8, 40)
    assert res.breakdown_dim == 12 and res.steps == 1
    assert np.linalg.norm(v - sector_evolve(H, v0, 20.0, [sec])) <= 1e-8


# ------------------------------------------------------------ trivial, aliasing, errors
def test_trivial_inputs_and_aliasing():
    announce("trivial")
    import torch
    te = lib()
    H, v0 = W.xxz_chain(9, seed=1)
    with hamiltonian(H) as h:
        x = to_dev(v0)
        out, res = te.te_evolve(h, x, 0.0, 1e-8, 20)
        assert torch.equal(out, x) and res.steps == 0
        z = torch.zeros_like(x)
        out, res = te.te_evolve(h, z, 3.0, 1e-8, 20)
        assert not torch.any(out) and res.err_bound == 0
        y = to_dev(2.0 * v0)
        ref, r1 = te.te_evolve(h, to_dev(v0), 3.0, 1e-8, 20)
        te.te_evolve(h, y, 3.0, 1e-8, 20, out=y)  # in place
        assert np.abs(to_host(y) - 2.0 * to_host(ref)).max() <= 1e-14


def test_determinism_bitwise():
    announce("determinism")
    te = lib()
    wl = W.workload("xxz_L12")
    with hamiltonian(wl.H) as h:
        a, _ = te.te_evolve(h, to_dev(wl.v0), wl.t, wl.tol, wl.m)
        b, _ = te.te_evolve(h, to_dev(wl.v0), wl.t, wl.tol, wl.m)
    assert np.array_equal(to_host(a), to_host(b))


def test_error_paths():
    announce("errors")
    te = lib()
    H, v0 = W.xxz_chain(6, seed=1)
    bad_rp = H.row_ptr.copy()
    bad_rp[3] = bad_rp[4] + 1
    for rp, ci, code in [(bad_rp, H.col, te.TE_ERR_INVALID_CSR),
                         (H.row_ptr, np.where(H.col == 5, 64, H.col).astype(np.int32), te.TE_ERR_INVALID_CSR)]:
        with pytest.raises(te.TEError) as e:
            te.te_hamiltonian_create(rp, ci, H.val)
        assert e.value.status == code
    val = H.val.copy()
    val[1] += 0.5j
    with pytest.raises(te.TEError) as e:
        te.te_hamiltonian_create(H.row_ptr, H.col, val, check_hermitian=True)
    assert e.value.status == te.TE_ERR_NOT_HERMITIAN
    te.te_hamiltonian_create(H.row_ptr, H.col, H.val, check_hermitian=True).destroy()
    with hamiltonian(H) as h:
        x = to_dev(v0)
        for args, code in [((1.0, 1e-8, 65), te.TE_ERR_UNSUPPORTED), ((1.0, 1e-8, 1), te.TE_ERR_INVALID_ARG),
                           ((-1.0, 1e-8, 10), te.TE_ERR_INVALID_ARG), ((1.0, 0.0, 10), te.TE_ERR_INVALID_ARG)]:
            with pytest.raises(te.TEError) as e:
                te.te_evolve(h, x, *args)
            assert e.value.status == code
        nan = to_dev(np.where(np.arange(H.dim) == 3, np.nan, v0))
        with pytest.raises(te.TEError) as e:
            te.te_evolve(h, nan, 1.0, 1e-8, 10)
        assert e.value.status == te.TE_ERR_NONFINITE
        with pytest.raises(te.TEError) as e:
            te.te_evolve(h, x, 50.0, 1e-10, 3, options=te.te_default_options(t_init=50.0, max_halvings=0))
        assert e.value.status == te.TE_ERR_STEP_UNDERFLOW
        _, res = te.te_evolve(h, x, 1.0, 1e-8, 20, options=te.te_default_options(quad_max_level=1))
        assert res.warnings & te.TE_WARN_QUADRATURE
        _, res = te.te_evolve(h, x, 1.0, 1e-15, 20)
        assert res.warnings & te.TE_WARN_NUMERICAL
        # the handle still works after errors
        v, res = te.te_evolve(h, x, 2.0, 1e-8, 20)
        assert res.err_bound <= 1e-8


# ------------------------------------------------------------------- autotuned kernel shapes
SHAPES = [(4, 1, 1, 1, 0), (4, 4, 1, 1, 0), (8, 2, 1, 1, 0), (4, 1, 2, 2, 0), (4, 4, 2, 2, 0), (8, 2, 2, 2, 0),
          (8, 2, 1, 2, 0), (4, 4, 1, 1, 1), (8, 2, 2, 2, 1), (4, 1, 2, 1, 1), (4, 4, 4, 1, 0), (8, 2, 4, 2, 1),
          (4, 1, 4, 2, 1), (1, 8, 4, 2, 0), (1, 8, 4, 2, 1), (1, 16, 4, 2, 0), (2, 8, 2, 2, 0)]


@pytest.mark.parametrize("shape", SHAPES)
def test_every_kernel_shape_matches_oracle(shape):
    announce(f"shape {shape}")
    te = lib()
    for H, v0, t, tol, m in [(*W.xxz_chain(11, seed=3), 6.0, 1e-8, 30),
                              (random_hermitian_csr(1537, 0.006, 11), None, 3.0, 1e-9, 24)]:
        if v0 is None:
            v0 = W.random_state(np.random.default_rng(11), H.dim)
        with hamiltonian(H) as h:
            te.te_set_tuning(h, *shape)
            got = te.te_get_tuning(h)
            assert (got.lanes_per_row, got.nnz_per_lane, got.rows_per_thread, got.update_rows_per_thread,
                    got.split_projection) == shape
            v, res = te.te_evolve(h, to_dev(v0), t, tol, m)
            v = to_host(v)
        ro = O.evolve(H, v0, t, tol, m)
        assert np.linalg.norm(v - ro.v) <= 2 * tol + 1e-12
        assert abs(res.steps - ro.steps) <= 1


@pytest.mark.parametrize("shape", [(4, 4, 1, 1), (8, 2, 2, 2), (4, 1, 2, 1), (8, 2, 4, 2), (1, 8, 4, 2)])
def test_split_projection_is_bitwise_the_fused_one(shape):
    """Sparse product and projections as two launches (y read back from memory) accumulate in
    the same order as the fused kernel: identical results."""
    announce(f"split vs fused {shape}")
    te = lib()
    H, v0 = W.xxz_chain(13, seed=5)
    out = []
    with hamiltonian(H) as h:
        x = to_dev(v0)
        for split in (0, 1):
            te.te_set_tuning(h, *shape, split)
            v, res = te.te_evolve(h, x, 7.0, 1e-8, 40)
            out.append((to_host(v), res.steps, res.err_bound))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1:] == out[1][1:]


def test_autotune_picks_a_supported_shape():
    announce("autotune")
    te = lib()
    wl = W.workload("xxz_L12")
    with hamiltonian(wl.H) as h:
        t = te.te_autotune(h, 40)
        assert (t.lanes_per_row, t.nnz_per_lane) in [(4, 1), (4, 4), (8, 2), (2, 8), (1, 8), (1, 16)]
        assert t.rows_per_thread in (1, 2, 4) and t.project_us > 0
        v, res = te.te_evolve(h, to_dev(wl.v0), wl.t, wl.tol, wl.m)
    ro = O.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m)
    assert np.linalg.norm(to_host(v) - ro.v) <= 2 * wl.tol + 1e-12
    with pytest.raises(te.TEError):
        with hamiltonian(wl.H) as h:
            te.te_set_tuning(h, 8, 4, 1, 1)
