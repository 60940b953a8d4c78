"""Storage kinds of H on the device (te_hamiltonian_create): packed entries (a 1- or 2-byte
code per entry into a table of (column - row, value) pairs, real diagonal per row), real
entries (8-byte values) and complex entries, each with the CSR's order of entries.  Every kind
computes the same products in the same order, so every result is compared bitwise across the
kinds, and against the oracle.  Matrices: the phase-twisted XXZ ring (complex, 2 pairs per
bond: 1-byte codes), its real part (real symmetric), the paper's own model (real), the Bose
chain (complex, hundreds of pairs: 2-byte codes), random Hermitian matrices (2-byte codes, or
too many pairs to pack), random patterns with few values (too many pairs, value codes beside
the columns), the paper's model built on the device and packed afterwards."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import few_values_hermitian, random_hermitian_csr
from tests.gpu_util import announce, lib, to_dev, to_host, torch_dev
from workloads.csr import CSR

pytestmark = pytest.mark.gpu


def real_xxz(L, seed, n_v0=1):
    H, v = W.xxz_chain(L, seed, n_v0=n_v0)
    return CSR(H.dim, H.row_ptr, H.col, np.ascontiguousarray(H.val.real.astype(np.complex128)), H.name + "_re"), v


def kinds(H):
    """The matrix as packed (default), CSR with real entries where possible, complex CSR."""
    te = lib()
    return [te.te_hamiltonian_create(H.row_ptr, H.col, H.val),
            te.te_hamiltonian_create(H.row_ptr, H.col, H.val, store_csr=True),
            te.te_hamiltonian_create(H.row_ptr, H.col, H.val, store_csr=True, store_complex=True)]


def destroy(*hs):
    for h in hs:
        h.destroy()


def roundtrip(te, h, H):
    rp, ci, va = te.te_hamiltonian_copy_csr(h)
    return (np.array_equal(rp, H.row_ptr) and np.array_equal(ci, H.col)
            and np.array_equal(va.view(np.float64), H.val.view(np.float64)))


def test_storage_detection():
    announce("storage detection")
    te = lib()
    H, _ = real_xxz(10, seed=1)
    hs = kinds(H)
    assert [h.storage for h in hs] == ["packed8", "real", "complex"]
    assert hs[1].real_values and not hs[0].real_values and not hs[2].real_values
    assert len({h.norm1 for h in hs}) == 1 and len({h.nnz for h in hs}) == 1
    assert all(roundtrip(te, h, H) for h in hs)
    Hx, _ = W.xxz_chain(10, seed=1)
    hx = kinds(Hx)
    assert [h.storage for h in hx] == ["packed8", "complex", "complex"]
    assert all(roundtrip(te, h, Hx) for h in hx)
    B, _ = W.bosonic_chain(8, 5, 3)
    hb = te.te_hamiltonian_create(B.row_ptr, B.col, B.val)
    assert hb.storage == "packed16" and roundtrip(te, hb, B)
    R = random_hermitian_csr(300, 0.03, seed=2)
    hr = te.te_hamiltonian_create(R.row_ptr, R.col, R.val)
    assert hr.storage == "packed16" and roundtrip(te, hr, R)
    # more than 65535 distinct pairs and values: CSR
    Rb = random_hermitian_csr(3000, 0.01, seed=3)
    hrb = te.te_hamiltonian_create(Rb.row_ptr, Rb.col, Rb.val)
    assert hrb.storage == "complex" and roundtrip(te, hrb, Rb)
    # more than 65535 pairs, few values: value codes beside the columns
    for n_values, kind in ((40, "coded8"), (2000, "coded16")):
        F = few_values_hermitian(3000, 0.01, 5, n_values)
        hf = te.te_hamiltonian_create(F.row_ptr, F.col, F.val, check_hermitian=True)
        assert hf.storage == kind and roundtrip(te, hf, F)
        hf.destroy()
    # one tiny imaginary pair: still packed, values kept bit for bit
    val = H.val.copy()
    rows = np.repeat(np.arange(H.dim), np.diff(H.row_ptr))
    off = np.flatnonzero(rows != H.col)[0]
    r, c = rows[off], H.col[off]
    back = H.row_ptr[c] + np.flatnonzero(H.col[H.row_ptr[c]:H.row_ptr[c + 1]] == r)[0]
    val[off] += 1e-300j
    val[back] -= 1e-300j
    Hi = CSR(H.dim, H.row_ptr, H.col, val, "tiny_imag")
    hi = te.te_hamiltonian_create(Hi.row_ptr, Hi.col, Hi.val, check_hermitian=True)
    hic = te.te_hamiltonian_create(Hi.row_ptr, Hi.col, Hi.val, store_csr=True)
    assert hi.storage == "packed8" and hic.storage == "complex" and roundtrip(te, hi, Hi)
    # device-pointer creation packs the same way
    import torch
    dev = torch_dev()
    hd = te.te_hamiltonian_create(torch.from_numpy(H.row_ptr).to(dev), torch.from_numpy(H.col).to(dev),
                                  torch.from_numpy(H.val).to(dev))
    assert hd.storage == "packed8" and roundtrip(te, hd, H)
    destroy(*hs, *hx, hb, hr, hrb, hi, hic, hd)


def test_diagonals_that_do_not_pack():
    """A complex or negative-zero imaginary diagonal, or a row storing its diagonal twice (no
    sorted-column check), keeps the CSR."""
    announce("diagonals that keep the CSR")
    te = lib()
    H, _ = W.xxz_chain(8, seed=4)
    rows = np.repeat(np.arange(H.dim), np.diff(H.row_ptr))
    dg = np.flatnonzero(rows == H.col)
    val = H.val.copy()
    val[dg[3]] = complex(val[dg[3]].real, 0.5)
    h = te.te_hamiltonian_create(H.row_ptr, H.col, val)
    assert h.storage == "complex" and roundtrip(te, h, CSR(H.dim, H.row_ptr, H.col, val, "d"))
    h.destroy()
    # -0.0 compares equal to zero: the real part alone is kept
    R, _ = real_xxz(8, seed=4)
    val = R.val.copy()
    val[dg[3]] = complex(val[dg[3]].real, -0.0)
    h = te.te_hamiltonian_create(R.row_ptr, R.col, val)
    assert h.storage == "real"
    h.destroy()
    # row 5 stores its diagonal twice (its first off-diagonal column rewritten to 5)
    col = H.col.copy()
    k = next(k for k in range(H.row_ptr[5], H.row_ptr[6]) if col[k] != 5)
    col[k] = 5
    h = te.te_hamiltonian_create(H.row_ptr, col, H.val)
    assert h.storage == "complex"
    h.destroy()


@pytest.mark.parametrize("shape", [(4, 4, 1, 1, 0), (8, 2, 4, 2, 1), (4, 1, 2, 1, 1), (8, 2, 2, 2, 0),
                                   (4, 4, 4, 2, 1), (2, 8, 2, 2, 1), (1, 8, 4, 2, 1), (1, 16, 4, 2, 0),
                                   (1, 8, 1, 1, 0), (1, 8, 4, 2, 0)])
@pytest.mark.parametrize("real", [False, True])
def test_evolve_is_bitwise_across_storage(shape, real):
    announce(f"evolution across storage, shape {shape}, real {real}")
    te = lib()
    H, v0 = real_xxz(13, seed=7) if real else W.xxz_chain(13, seed=7)
    hs = kinds(H)
    x = to_dev(v0)
    out = []
    for h in hs:
        te.te_set_tuning(h, *shape)
        v, res = te.te_evolve(h, x, 9.0, 1e-8, 40)
        out.append((to_host(v), res.steps, res.matvecs, res.err_bound, res.num_err_estimate))
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0]) and out[0][1:] == o[1:]
    ro = O.evolve(H, v0, 9.0, 1e-8, 40)
    assert np.linalg.norm(out[0][0] - ro.v) <= 2e-8 + 1e-12
    destroy(*hs)


@pytest.mark.parametrize("n_values", [40, 2000])
@pytest.mark.parametrize("shape", [(4, 4, 2, 2, 1), (1, 8, 4, 2, 1), (8, 2, 1, 1, 0), (1, 16, 2, 2, 0),
                                   (1, 8, 4, 2, 0)])
def test_value_codes_evolve_bitwise_and_match_oracle(shape, n_values):
    announce(f"value codes ({n_values} values), shape {shape}")
    te = lib()
    H = few_values_hermitian(3000, 0.01, 5, n_values)
    v0 = W.random_state(np.random.default_rng(6), H.dim)
    hs = kinds(H)
    assert [h.storage for h in hs] == ["coded8" if n_values < 128 else "coded16", "complex", "complex"]
    x = to_dev(v0)
    out = []
    for h in hs[:2]:
        te.te_set_tuning(h, *shape)
        v, res = te.te_evolve(h, x, 1.5, 1e-8, 30)
        out.append((to_host(v), res.steps, res.err_bound))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    ro = O.evolve(H, v0, 1.5, 1e-8, 30)
    assert np.linalg.norm(out[0][0] - ro.v) <= 2e-8 + 1e-12
    destroy(*hs)


def test_packing_a_device_built_matrix():
    """te_hamiltonian_pack on the paper's model built on the device (real CSR): at the Fig. 1
    size its pairs pack; with 20 memory qubits and 5 excitations they are too many and its
    couplings become value codes.  Evolutions are bitwise those of the unpacked handle."""
    announce("packing device-built matrices")
    te = lib()
    for params, kind in ((dict(), "packed8"), (dict(K=10, Kp=10, N0=10, Nm=5), "coded8")):
        h, idx = te.te_hamiltonian_create_memory_burden(**params)
        assert h.storage == "real"
        v0 = np.zeros(h.dim, dtype=np.complex128)
        v0[idx] = 1.0
        x = to_dev(v0)
        out = []
        # evolve as CSR (the handle's restart graph is captured on the CSR arrays), pack, evolve
        # again with the same shape: the packed products are bitwise the CSR ones
        te.te_set_tuning(h, 4, 4, 2, 2, 1)
        v, res = te.te_evolve(h, x, 2.0, 1e-8, 40)
        out.append((to_host(v), res.steps, res.err_bound))
        rp0, ci0, va0 = te.te_hamiltonian_copy_csr(h)
        assert te.te_hamiltonian_pack(h) == kind and h.storage == kind
        assert te.te_hamiltonian_pack(h) == kind  # no-op when packed
        rp1, ci1, va1 = te.te_hamiltonian_copy_csr(h)
        assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1) and np.array_equal(va0, va1)
        te.te_set_tuning(h, 4, 4, 2, 2, 1)
        v, res = te.te_evolve(h, x, 2.0, 1e-8, 40)
        out.append((to_host(v), res.steps, res.err_bound))
        assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
        h.destroy()


@pytest.mark.parametrize("shape", [(4, 4, 2, 2, 1), (1, 8, 4, 2, 1), (2, 8, 2, 2, 0), (1, 8, 4, 2, 0)])
def test_two_byte_codes_evolve_bitwise_and_match_oracle(shape):
    announce(f"2-byte codes: Bose chain, shape {shape}")
    te = lib()
    H, v0 = W.bosonic_chain(8, 5, 3)
    hs = kinds(H)
    assert [h.storage for h in hs] == ["packed16", "complex", "complex"]
    x = to_dev(v0)
    out = []
    for h in hs[:2]:
        te.te_set_tuning(h, *shape)
        v, res = te.te_evolve(h, x, 5.0, 1e-9, 30)
        out.append((to_host(v), res.steps, res.err_bound))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    ro = O.evolve(H, v0, 5.0, 1e-9, 30)
    assert np.linalg.norm(out[0][0] - ro.v) <= 2e-9 + 1e-12
    destroy(*hs)


def test_spmv_is_bitwise_across_storage():
    announce("te_spmv across storage")
    te = lib()
    H, _, _ = W.memory_burden_model(K=4, Kp=4, Nm=2, N0=6)
    hs = kinds(H)
    assert [h.storage for h in hs] == ["packed8", "real", "complex"]
    x = to_dev(W.random_state(np.random.default_rng(4), H.dim))
    ys = [te.te_spmv(h, x) for h in hs]
    for y, d in ys[1:]:
        assert np.array_equal(to_host(ys[0][0]), to_host(y)) and ys[0][1] == d
    ref = H.to_scipy() @ to_host(x)
    assert np.max(np.abs(to_host(ys[0][0]) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    destroy(*hs)


def test_paper_model_matches_oracle_in_every_storage():
    announce("paper model across storage")
    te = lib()
    H, v0, _ = W.memory_burden_model(K=5, Kp=5, Nm=3, N0=8)
    hs = kinds(H)
    assert [h.storage for h in hs] == ["packed16", "real", "complex"]
    x = to_dev(v0)
    ro = O.evolve(H, v0, 10.0, 1e-8, 40)
    for shape in ((4, 4, 2, 2, 0), (1, 8, 4, 2, 1)):  # the lanes per row fix the order of the sums
        res = []
        for h in hs:
            te.te_set_tuning(h, *shape)
            res.append(te.te_evolve(h, x, 10.0, 1e-8, 40))
        for v, r in res[1:]:
            assert np.array_equal(to_host(res[0][0]), to_host(v)) and res[0][1].err_bound == r.err_bound
        assert np.linalg.norm(to_host(res[0][0]) - ro.v) <= 2e-8 + 1e-12
    destroy(*hs)


def test_batch_mixes_storage_kinds():
    """One round graph holds groups of every kind (fused single-vector groups and multi-vector
    products); every job's result is bitwise its result alone."""
    announce("batch across storage kinds")
    te = lib()
    H, vs = real_xxz(11, seed=9, n_v0=3)
    hp, hr, hc = kinds(H)
    R = few_values_hermitian(3000, 0.01, 10, 40)
    hz = te.te_hamiltonian_create(R.row_ptr, R.col, R.val)
    assert hz.storage == "coded8"
    rv = [W.random_state(np.random.default_rng(11), 3000)]
    groups = [(hp, [to_dev(v) for v in vs], 6.0, 1e-8), (hr, [to_dev(v) for v in vs], 6.0, 1e-8),
              (hc, [to_dev(v) for v in vs], 6.0, 1e-8), (hp, [to_dev(vs[0])], 4.0, 1e-8),
              (hz, [to_dev(v) for v in rv], 3.0, 1e-8)]
    outs, results, st = te.te_batch_run(groups, m=40, shape=(4, 4), rows_per_thread=2, update_rows_per_thread=2)
    assert st.jobs_done == 11 and st.jobs_failed == 0
    for q in range(3):
        assert np.array_equal(to_host(outs[0][q]), to_host(outs[1][q]))
        assert np.array_equal(to_host(outs[0][q]), to_host(outs[2][q]))
    for q, (r, s, _) in enumerate(results[:3]):
        assert s == te.TE_OK and (r.steps, r.err_bound) == (results[3 + q][0].steps, results[3 + q][0].err_bound)
    for h, v, t, o in ((hp, vs[0], 4.0, outs[3][0]), (hz, rv[0], 3.0, outs[4][0])):
        te.te_set_tuning(h, 4, 4, 2, 2, 0)
        ref, _ = te.te_evolve(h, to_dev(v), t, 1e-8, 40)
        assert np.array_equal(to_host(ref), to_host(o))
    ro = O.evolve(H, vs[1], 6.0, 1e-8, 40)
    assert np.linalg.norm(to_host(outs[0][1]) - ro.v) <= 2e-8 + 1e-12
    destroy(hp, hr, hc, hz)


def column_bytes_per_entry(te, h_coded, h_csr, H, x, shape):
    """Bytes per entry the library's byte model charges the value-coded columns, from the
    projection bytes of the same evolution on the coded and the complex-CSR handle: per launch
    the coded matrix moves (1 + c) nnz + 8 d bytes where the CSR moves 20 nnz."""
    prof = te.te_default_options(flags=te.TE_OPT_PROFILE)
    got = []
    for h in (h_coded, h_csr):
        te.te_set_tuning(h, *shape)
        v, res = te.te_evolve(h, x, 0.5, 1e-8, 20, options=prof)
        p = te.te_last_profile(h).as_dict()["project"]
        got.append((p["bytes"], p["launches"], to_host(v), res.steps))
    (b0, n0, v0, s0), (b1, n1, v1, s1) = got
    assert n0 == n1 and s0 == s1 and np.array_equal(v0, v1)  # same launches, bitwise the same result
    return ((b0 - b1) / n0 - 8.0 * H.dim + 19.0 * H.nnz) / H.nnz


@pytest.mark.parametrize("shape", [(1, 8, 4, 2, 1), (1, 8, 4, 2, 0)])
def test_value_code_columns_16_and_32_bit(shape):
    """Value codes keep each column as a 16-bit offset from a base per group (the entries q of a
    chunk of 64 rows) when every group spans at most 65535 columns, else as 32 bits.  Both forms
    expand back to the uploaded CSR and evolve bitwise like it."""
    announce(f"value-code columns, 16 and 32 bit, shape {shape}")
    te = lib()
    # narrow: 3000 rows, every group within 3000 columns
    N = few_values_hermitian(3000, 0.01, 5, 40)
    # wide: 70000 rows with random columns, groups spanning nearly the whole range
    Wd = few_values_hermitian(70000, 5e-5, 7, 40)
    for H, want in ((N, 2.0), (Wd, 4.0)):
        hc = te.te_hamiltonian_create(H.row_ptr, H.col, H.val)
        hx = te.te_hamiltonian_create(H.row_ptr, H.col, H.val, store_csr=True, store_complex=True)
        try:
            assert hc.storage == "coded8" and hx.storage == "complex"
            assert roundtrip(te, hc, H)
            v0 = W.random_state(np.random.default_rng(11), H.dim)
            assert column_bytes_per_entry(te, hc, hx, H, to_dev(v0), shape) == pytest.approx(want, abs=1e-9)
        finally:
            destroy(hc, hx)
