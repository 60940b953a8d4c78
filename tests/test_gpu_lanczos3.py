"""Three-term mode (TE_OPT_LANCZOS3: step 1 with the recurrence as printed in eq. arnoldi /
Alg. 1, no re-orthogonalisation) through the C ABI, against the oracle's three-term mode and
exact answers.  Without re-orthogonalisation rounding differences grow with j, so the bar is
the one both sides satisfy against the exact answer: ||v_gpu - v_oracle|| <= 2 tol + 1e-12,
and each result within its own bound of the exact answer where one is available."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import dense_evolve, random_hermitian_csr, sector_evolve, xxz_sectors
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu


def opts3(te, **kw):
    return te.te_default_options(flags=te.TE_OPT_LANCZOS3, **kw)


@pytest.mark.parametrize("case", ["xxz_L12", "rand700", "bose6", "xxz10_m64"])
def test_three_term_matches_oracle(case):
    announce(f"three-term {case}")
    te = lib()
    if case == "xxz_L12":
        wl = W.workload("xxz_L12")
        H, v0, t, tol, m = wl.H, wl.v0, wl.t, wl.tol, wl.m
        exact = sector_evolve(H, v0, t, xxz_sectors(12))
    elif case == "rand700":
        H = random_hermitian_csr(700, 0.02, 61)
        v0 = W.random_state(np.random.default_rng(62), 700)
        t, tol, m = 4.0, 1e-9, 30
        exact = dense_evolve(H, v0, t)
    elif case == "bose6":
        H, v0 = W.bosonic_chain(6, 6, seed=63)
        t, tol, m = 5.0, 1e-8, 40
        exact = None
    else:
        H, v0 = W.xxz_chain(10, seed=64)
        t, tol, m = 20.0, 1e-8, 64
        exact = dense_evolve(H, v0, t)
    with hamiltonian(H) as h:
        v, res = te.te_evolve(h, to_dev(v0), t, tol, m, options=opts3(te))
        v = to_host(v)
    ro = O.evolve(H, v0, t, tol, m, three_term=True)
    assert np.linalg.norm(v - ro.v) <= 2 * tol + 1e-12
    assert res.err_bound <= tol * (1 + 1e-12)
    if exact is not None:
        assert np.linalg.norm(v - exact) <= res.err_bound * (1 + 1e-3) + 1e-12


def test_three_term_kernel_shapes_agree_bitwise():
    announce("three-term shapes")
    te = lib()
    H, v0 = W.xxz_chain(13, seed=65)
    outs = []
    with hamiltonian(H) as h:
        x = to_dev(v0)
        for shape in [(4, 4, 1, 1, 0), (4, 4, 1, 1, 1), (8, 2, 2, 2, 0), (8, 2, 2, 2, 1), (8, 2, 4, 2, 0),
                      (8, 2, 4, 2, 1)]:
            te.te_set_tuning(h, *shape)
            v, res = te.te_evolve(h, x, 6.0, 1e-8, 40, options=opts3(te))
            outs.append((shape, to_host(v), res.steps))
    # split and fused forms of one shape are bitwise equal; other shapes within the bounds
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[2][1], outs[3][1])
    assert np.array_equal(outs[4][1], outs[5][1])
    assert np.linalg.norm(outs[0][1] - outs[2][1]) <= 2e-8 + 1e-12


def test_three_term_moves_fewer_bytes_on_the_bench_matrix():
    """XXZ L=20 (d = 2^20): the three-term build reads 2 basis columns per pass instead of j + 1;
    the bound still holds (norm conservation within it) and the profile's algorithmic bytes
    per restart drop accordingly."""
    announce("three-term L=20")
    te = lib()
    wl = W.workload("xxz_L20")
    with hamiltonian(wl.H) as h:
        x = to_dev(wl.v0)
        prof = te.te_default_options(flags=te.TE_OPT_PROFILE | te.TE_OPT_LANCZOS3)
        v3, r3 = te.te_evolve(h, x, 10.0, wl.tol, wl.m, options=prof)
        p3 = te.te_last_profile(h).as_dict()
        vf, rf = te.te_evolve(h, x, 10.0, wl.tol, wl.m, options=te.te_default_options(flags=te.TE_OPT_PROFILE))
        pf = te.te_last_profile(h).as_dict()
        assert r3.err_bound <= wl.tol and rf.err_bound <= wl.tol
        assert abs(float(v3.norm()) - 1.0) <= r3.err_bound + 1e-10
        assert float((v3 - vf).norm()) <= r3.err_bound + rf.err_bound + 1e-10
    per3 = (p3["project"]["bytes"] + p3["update"]["bytes"]) / r3.steps
    perf = (pf["project"]["bytes"] + pf["update"]["bytes"]) / rf.steps
    assert perf / per3 > 2.5


def test_engine_three_term_equals_alone():
    announce("engine three-term")
    te = lib()
    H, vs = W.xxz_chain(11, seed=66, n_v0=3)
    with hamiltonian(H) as h:
        dev = [to_dev(v) for v in vs]
        outs, results, st = te.te_batch_run([(h, dev, 7.0, 1e-8)], m=40, shape=(4, 4), rows_per_thread=2,
                                            update_rows_per_thread=2, options=opts3(te))
        te.te_set_tuning(h, 4, 4, 2, 2, 0)
        for d, o, (res, status, _) in zip(dev, outs[0], results):
            assert status == te.TE_OK
            ref, rres = te.te_evolve(h, d, 7.0, 1e-8, 40, options=opts3(te))
            assert bool((o == ref).all())
            assert res.steps == rres.steps and res.err_bound == rres.err_bound
