"""Real-entry storage of H: a matrix whose imaginary parts are all zero keeps 8-byte entries on
the device.  The sparse products then compute the same values as with the complex copy (the
zero imaginary parts only add exact zeros), so every result is compared bitwise with the same
matrix held as complex (TE_STORE_COMPLEX), and against the oracle.  Real matrices: the paper's
own model (real coefficients) and the real part of the XXZ ring (Re H is symmetric for
Hermitian H; the phase-twisted ring itself is complex)."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import random_hermitian_csr
from tests.gpu_util import announce, lib, to_dev, to_host, torch_dev
from workloads.csr import CSR

pytestmark = pytest.mark.gpu


def real_xxz(L, seed, n_v0=1):
    H, v = W.xxz_chain(L, seed, n_v0=n_v0)
    return CSR(H.dim, H.row_ptr, H.col, np.ascontiguousarray(H.val.real.astype(np.complex128)), H.name + "_re"), v


def both(H):
    te = lib()
    hr = te.te_hamiltonian_create(H.row_ptr, H.col, H.val)
    hc = te.te_hamiltonian_create(H.row_ptr, H.col, H.val, store_complex=True)
    return hr, hc


def test_storage_follows_the_imaginary_parts():
    announce("storage detection")
    te = lib()
    H, _ = real_xxz(10, seed=1)
    hr, hc = both(H)
    assert hr.real_values and not hc.real_values
    Hx, _ = W.xxz_chain(10, seed=1)
    assert not te.te_hamiltonian_create(Hx.row_ptr, Hx.col, Hx.val).real_values
    assert hr.norm1 == hc.norm1 and hr.nnz == hc.nnz
    R = random_hermitian_csr(300, 0.03, seed=2)
    assert not te.te_hamiltonian_create(R.row_ptr, R.col, R.val).real_values
    # one tiny imaginary pair keeps the complex copy
    val = H.val.copy()
    rows = np.repeat(np.arange(H.dim), np.diff(H.row_ptr))
    off = np.flatnonzero(rows != H.col)[0]
    r, c = rows[off], H.col[off]
    back = H.row_ptr[c] + np.flatnonzero(H.col[H.row_ptr[c]:H.row_ptr[c + 1]] == r)[0]
    val[off] += 1e-300j
    val[back] -= 1e-300j
    hi = te.te_hamiltonian_create(H.row_ptr, H.col, val, check_hermitian=True)
    assert not hi.real_values
    # device-pointer creation detects it the same way
    import torch
    dev = torch_dev()
    hd = te.te_hamiltonian_create(torch.from_numpy(H.row_ptr).to(dev), torch.from_numpy(H.col).to(dev),
                                  torch.from_numpy(H.val).to(dev))
    assert hd.real_values
    for h in (hr, hc, hi, hd):
        h.destroy()


@pytest.mark.parametrize("shape", [(4, 4, 1, 1, 0), (8, 2, 4, 2, 1), (4, 1, 2, 1, 1), (8, 2, 2, 2, 0)])
def test_evolve_real_storage_is_bitwise_the_complex_one(shape):
    announce(f"real vs complex storage, shape {shape}")
    te = lib()
    H, v0 = real_xxz(13, seed=7)
    hr, hc = both(H)
    x = to_dev(v0)
    out = []
    for h in (hr, hc):
        te.te_set_tuning(h, *shape)
        v, res = te.te_evolve(h, x, 9.0, 1e-8, 40)
        out.append((to_host(v), res.steps, res.matvecs, res.err_bound, res.num_err_estimate))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    ro = O.evolve(H, v0, 9.0, 1e-8, 40)
    assert np.linalg.norm(out[0][0] - ro.v) <= 2e-8 + 1e-12
    hr.destroy()
    hc.destroy()


def test_spmv_real_storage_is_bitwise_the_complex_one():
    announce("te_spmv real vs complex storage")
    te = lib()
    H, _, _ = W.memory_burden_model(K=4, Kp=4, Nm=2, N0=6)
    hr, hc = both(H)
    assert hr.real_values
    x = to_dev(W.random_state(np.random.default_rng(4), H.dim))
    yr, dr = te.te_spmv(hr, x)
    yc, dc = te.te_spmv(hc, x)
    assert np.array_equal(to_host(yr), to_host(yc)) and dr == dc
    ref = H.to_scipy() @ to_host(x)
    assert np.max(np.abs(to_host(yr) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    hr.destroy()
    hc.destroy()


def test_paper_model_real_storage_matches_oracle():
    announce("paper model, real storage")
    te = lib()
    H, v0, _ = W.memory_burden_model(K=5, Kp=5, Nm=3, N0=8)
    hr, hc = both(H)
    assert hr.real_values
    x = to_dev(v0)
    vr, rr = te.te_evolve(hr, x, 10.0, 1e-8, 40)
    vc, rc = te.te_evolve(hc, x, 10.0, 1e-8, 40)
    assert np.array_equal(to_host(vr), to_host(vc)) and rr.err_bound == rc.err_bound
    ro = O.evolve(H, v0, 10.0, 1e-8, 40)
    assert np.linalg.norm(to_host(vr) - ro.v) <= 2e-8 + 1e-12
    hr.destroy()
    hc.destroy()


def test_batch_mixes_real_and_complex_storage():
    """One round graph holds groups of both kinds (fused single-vector groups and multi-vector
    products); every job's result is bitwise its result alone with the same storage."""
    announce("batch with real and complex storage")
    te = lib()
    H, vs = real_xxz(11, seed=9, n_v0=3)
    hr, hc = both(H)
    R = random_hermitian_csr(900, 0.02, seed=10)
    hz = te.te_hamiltonian_create(R.row_ptr, R.col, R.val)
    rv = [W.random_state(np.random.default_rng(11), 900)]
    groups = [(hr, [to_dev(v) for v in vs], 6.0, 1e-8), (hc, [to_dev(v) for v in vs], 6.0, 1e-8),
              (hr, [to_dev(vs[0])], 4.0, 1e-8), (hz, [to_dev(v) for v in rv], 3.0, 1e-8)]
    outs, results, st = te.te_batch_run(groups, m=40, shape=(4, 4), rows_per_thread=2, update_rows_per_thread=2)
    assert st.jobs_done == 8 and st.jobs_failed == 0
    for a, b in ((outs[0][q], outs[1][q]) for q in range(3)):
        assert np.array_equal(to_host(a), to_host(b))
    for q, (r, s, _) in enumerate(results[:3]):
        assert s == te.TE_OK and (r.steps, r.err_bound) == (results[3 + q][0].steps, results[3 + q][0].err_bound)
    for h, v, t, o in ((hr, vs[0], 4.0, outs[2][0]), (hz, rv[0], 3.0, outs[3][0])):
        te.te_set_tuning(h, 4, 4, 2, 2, 0)
        ref, _ = te.te_evolve(h, to_dev(v), t, 1e-8, 40)
        assert np.array_equal(to_host(ref), to_host(o))
    ro = O.evolve(H, vs[1], 6.0, 1e-8, 40)
    assert np.linalg.norm(to_host(outs[0][1]) - ro.v) <= 2e-8 + 1e-12
    for h in (hr, hc, hz):
        h.destroy()
