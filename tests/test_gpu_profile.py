"""Profiling mode of te_evolve (TE_OPT_PROFILE): per-kernel timing events are bound to the
dispatches of directly launched restarts.  The solve must be bitwise the one the restart graphs
(and plain direct launches) give, and the profile's launch counts, algorithmic bytes and
durations must account for the whole solve."""

import os
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import announce, lib, to_dev, to_host
from workloads.csr import CSR

pytestmark = pytest.mark.gpu

M = 40


def _evolve(te, h, x, t, tol, flags=0):
    opts = te.te_default_options(flags=flags) if flags else None
    v, res = te.te_evolve(h, x, t, tol, M, options=opts)
    return to_host(v), (res.steps, res.matvecs, res.err_bound, res.num_err_estimate)


def expected_project_bytes(H, kind, steps):
    d, nnz = float(H.dim), float(H.nnz)
    entries = {"complex": 20.0 * nnz, "real": 12.0 * nnz, "packed8": 1.0 * nnz + 8.0 * d}[kind]
    per_restart = sum(entries + 4.0 * (d + 1) + 16.0 * d * (j + 2) for j in range(M))
    return steps * per_restart


@pytest.mark.parametrize("kind", ["complex", "real", "packed8"])
def test_profiled_solve_is_bitwise_the_graph_solve(kind):
    announce(f"profile vs graph, storage {kind}")
    te = lib()
    H, v0 = W.xxz_chain(13, seed=31)
    if kind == "real":
        H = CSR(H.dim, H.row_ptr, H.col, np.ascontiguousarray(H.val.real.astype(np.complex128)), "xxz_re")
    with te.te_hamiltonian_create(H.row_ptr, H.col, H.val, store_csr=kind != "packed8") as h:
        assert h.storage == kind
        te.te_set_tuning(h, 8, 2, 4, 2, 1)
        x = to_dev(v0)
        vg, rg = _evolve(te, h, x, 12.0, 1e-8)
        t0 = time.perf_counter()
        vp, rp = _evolve(te, h, x, 12.0, 1e-8, te.TE_OPT_PROFILE)
        wall = time.perf_counter() - t0
        prof = te.te_last_profile(h).as_dict()
        os.environ["TE_NO_GRAPH"] = "1"
        try:
            vd, rd = _evolve(te, h, x, 12.0, 1e-8)
        finally:
            del os.environ["TE_NO_GRAPH"]
    assert np.array_equal(vg, vp) and rg == rp
    assert np.array_equal(vg, vd) and rg == rd
    steps, matvecs = rp[0], rp[1]
    # no breakdown at d = 8192: every restart runs m projections and updates
    assert prof["project"]["launches"] == steps * M == matvecs
    assert prof["update"]["launches"] == steps * M and prof["fold"]["launches"] == steps * M
    assert prof["step"]["launches"] == steps and prof["combine"]["launches"] == steps
    want = expected_project_bytes(H, kind, steps)
    assert prof["project"]["bytes"] == pytest.approx(want, rel=1e-12)
    secs = [prof[k]["seconds"] for k in te.KERNEL_CLASSES]
    assert all(s > 0 for s in secs)
    # the classes tile the solve's device time: their sum cannot exceed the host-measured call
    assert sum(secs) <= wall
