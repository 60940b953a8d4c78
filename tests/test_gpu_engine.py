"""Batched and served evolution (te_batch_*, te_engine_*) through the C ABI.

A job's arithmetic in the batched kernels is the arithmetic of te_evolve with the same kernel
shape (one row per thread in the projection, the same lanes per row, nonzeros in flight and
update rows per thread): results must be bitwise identical to the job run alone, whatever the
other jobs of the round are.  Against the CPU oracle the bar is that of the single-solve
parity tests, ||v_gpu - v_oracle|| <= 2 tol + 1e-12; results of different kernel shapes agree
within the sum of their error bounds (+1e-12)."""

import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.exact import random_hermitian_csr
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu
SHAPE = (4, 4)
TUNE = dict(shape=SHAPE, rows_per_thread=2, update_rows_per_thread=2)
M = 40


def alone(h, v0, t, tol, shape=SHAPE, rpt=2, rpt_u=2, m=M, split=0):
    te = lib()
    te.te_set_tuning(h, shape[0], shape[1], rpt, rpt_u, split)
    out, res = te.te_evolve(h, v0, t, tol, m)
    return out.clone(), res


def same_result(a, b):
    return (a.steps, a.matvecs, a.breakdown_dim, a.warnings, a.err_bound, a.num_err_estimate, a.t_reached) == \
        (b.steps, b.matvecs, b.breakdown_dim, b.warnings, b.err_bound, b.num_err_estimate, b.t_reached)


def xxz_group(L, seed, n, t, tol):
    H, vs = W.xxz_chain(L, seed, n_v0=n)
    vs = [vs] if n == 1 else vs
    return H, vs, t, tol


@pytest.fixture(scope="module")
def mixed_groups():
    groups = [xxz_group(10, 11, 3, 5.0, 1e-8), xxz_group(11, 12, 1, 3.0, 1e-6), xxz_group(12, 13, 2, 8.0, 1e-10)]
    R = random_hermitian_csr(700, 0.02, seed=14)
    rng = np.random.default_rng(15)
    groups.append((R, [W.random_state(rng, 700) for _ in range(2)], 2.0, 1e-8))
    Hb, vb = W.bosonic_chain(5, 5, seed=16)
    groups.append((Hb, [vb], 4.0, 1e-8))
    return groups


@pytest.mark.parametrize("tune", [((4, 4), 2, 2), ((8, 2), 1, 1), ((4, 1), 2, 1), ((8, 2), 4, 2), ((1, 8), 4, 2),
                                  ((1, 8), 1, 1)])
def test_batch_bitwise_equals_alone(mixed_groups, tune):
    te = lib()
    shape, rpt, rpt_u = tune
    hs = [hamiltonian(H) for H, _, _, _ in mixed_groups]
    dev = [[to_dev(v) for v in vs] for _, vs, _, _ in mixed_groups]
    announce(f"batch of 9 jobs on 5 Hamiltonians, shape {tune}")
    outs, results, stats = te.te_batch_run([(h, d, t, tol) for h, d, (_, _, t, tol) in zip(hs, dev, mixed_groups)],
                                           m=M, shape=shape, rows_per_thread=rpt, update_rows_per_thread=rpt_u)
    assert stats.jobs_done == 9 and stats.jobs_failed == 0
    assert stats.rounds >= max(r.steps for r, _, _ in results)
    i = 0
    for gi, (h, d, (_, _, t, tol)) in enumerate(zip(hs, dev, mixed_groups)):
        for vi, v in enumerate(d):
            announce(f"alone: group {gi} vector {vi}")
            ref, rres = alone(h, v, t, tol, shape=shape, rpt=rpt, rpt_u=rpt_u, split=vi % 2)
            res, status, _ = results[i]
            assert status == te.TE_OK
            assert same_result(res, rres), (gi, vi, res.as_dict(), rres.as_dict())
            assert bool((outs[gi][vi] == ref).all()), (gi, vi)
            i += 1
    for h in hs:
        h.destroy()


def test_batch_matches_oracle():
    te = lib()
    H, vs, t, tol = xxz_group(10, 31, 2, 10.0, 1e-8)
    announce("batch L=10 x2 vs oracle")
    with hamiltonian(H) as h:
        outs, results, _ = te.te_batch_run([(h, [to_dev(v) for v in vs], t, tol)], m=M)
        for v, o, (res, status, _) in zip(vs, outs[0], results):
            assert status == te.TE_OK
            ref = O.evolve(H, v, t, tol, M)
            assert np.linalg.norm(to_host(o) - ref.v) <= 2 * tol + 1e-12
            assert res.err_bound <= tol * (1 + 1e-12)


def test_batch_autotuned_agrees_with_alone(mixed_groups):
    te = lib()
    hs = [hamiltonian(H) for H, _, _, _ in mixed_groups]
    dev = [[to_dev(v) for v in vs] for _, vs, _, _ in mixed_groups]
    announce("batch autotuned")
    outs, results, stats = te.te_batch_run([(h, d, t, tol) for h, d, (_, _, t, tol) in zip(hs, dev, mixed_groups)],
                                           m=M)
    assert (stats.tuning.lanes_per_row, stats.tuning.nnz_per_lane) in [(4, 1), (4, 4), (8, 2), (1, 8)]
    assert stats.tuning.project_us > 0
    i = 0
    for gi, (h, d, (_, _, t, tol)) in enumerate(zip(hs, dev, mixed_groups)):
        for vi, v in enumerate(d):
            ref, rres = alone(h, v, t, tol, shape=(8, 2), rpt=1, rpt_u=1)
            res, status, _ = results[i]
            assert status == te.TE_OK
            err = float((outs[gi][vi] - ref).norm())
            assert err <= res.err_bound + rres.err_bound + 1e-12, (gi, vi, err)
            i += 1
    for h in hs:
        h.destroy()


def test_engine_alone_and_in_the_mix():
    """Continuous batching: the same request gives the same bits alone and when it arrives
    while other requests of several sizes are running."""
    te = lib()
    HA, vA = W.xxz_chain(12, 21, n_v0=3)
    HC, vC = W.xxz_chain(11, 22)
    HD, vD = W.bosonic_chain(6, 6, seed=23)
    budget = 6 * te.te_job_footprint(4096, M)
    with hamiltonian(HA) as hA, hamiltonian(HC) as hC, hamiltonian(HD) as hD:
        # B, C, D arrive together; A2 and E arrive while they run (B is long: t=100 at 1e-10)
        reqs = [("B", hA, vA[1], 100.0, 1e-10), ("C", hC, vC, 30.0, 1e-6), ("D", hD, vD, 10.0, 1e-8),
                ("A2", hA, vA[0], 20.0, 1e-8), ("E", hA, vA[2], 5.0, 1e-8)]
        dev = {name: to_dev(v) for name, _, v, _, _ in reqs}
        dev["A"] = dev["A2"]
        with te.Engine(budget, m=M, max_jobs=8, **TUNE) as eng:
            announce("engine: A alone")
            ja = eng.submit(hA, dev["A"], 20.0, 1e-8)
            eng.wait(ja, timeout=120)
            info, res_alone = eng.poll(ja)
            assert info.state == te.TE_JOB_DONE
            out_alone = eng.output(ja).clone()
            announce("engine: mix of 5 requests, two arriving while the others run")
            ids = {}
            for name, h, _, t, tol in reqs:
                if name == "A2":
                    time.sleep(0.005)
                ids[name] = eng.submit(h, dev[name], t, tol)
            eng.wait(-1, timeout=300)
            infos = {n: eng.poll(j) for n, j in ids.items()}
            for n, (info, res) in infos.items():
                assert info.state == te.TE_JOB_DONE, (n, info.as_dict())
            # the request is bitwise the same alone and in the mix
            assert bool((eng.output(ids["A2"]) == out_alone).all())
            assert same_result(infos["A2"][1], res_alone)
            # every request equals its own solo te_evolve run
            for name, h, _, t, tol in reqs:
                ref, rres = alone(h, dev[name], t, tol)
                assert bool((eng.output(ids[name]) == ref).all()), name
                assert same_result(infos[name][1], rres), name
            # A2 joined while B was running: admitted at a later round boundary, before B finished
            iB, iA2 = infos["B"][0], infos["A2"][0]
            assert iB.admitted < iA2.admitted < iB.finished, (iB.as_dict(), iA2.as_dict())
            assert iA2.rounds < iB.rounds
            st = eng.stats()
            assert st.pool_peak <= budget and st.jobs_done == 6 and st.plans >= 2


@pytest.mark.parametrize("threaded", [True, False])
def test_engine_two_lanes(threaded):
    """Two lanes: jobs of at least lane_rows rows run in their own lane (at most lane_jobs
    resident, in submission order), the others beside them; every result is bitwise its solo
    te_evolve run, ids follow submission order over both lanes, statistics add up."""
    te = lib()
    HL, vL = W.xxz_chain(13, 61, n_v0=3)   # 8192 rows: the large-job lane
    HS, vS = W.xxz_chain(10, 62, n_v0=2)   # 1024 rows: the small-job lane
    HB, vB = W.bosonic_chain(6, 6, seed=63)  # 462 rows
    budget = 2 * 4 * te.te_job_footprint(8192, M)
    with hamiltonian(HL) as hL, hamiltonian(HS) as hS, hamiltonian(HB) as hB:
        reqs = [(hL, vL[0], 20.0, 1e-8), (hS, vS[0], 40.0, 1e-10), (hL, vL[1], 5.0, 1e-8),
                (hB, vB, 30.0, 1e-10), (hL, vL[2], 10.0, 1e-6), (hS, vS[1], 3.0, 1e-8)]
        dev = [to_dev(v) for _, v, _, _ in reqs]
        announce(f"engine: two lanes, threaded={threaded}")
        with te.Engine(budget, m=M, max_jobs=8, threaded=threaded, lane_rows=4096, lane_jobs=1, **TUNE) as eng:
            ids = [eng.submit(h, d, t, tol) for (h, _, t, tol), d in zip(reqs, dev)]
            assert ids == list(range(len(reqs)))
            eng.wait(-1, timeout=300)
            infos = [eng.poll(j) for j in ids]
            assert all(i.state == te.TE_JOB_DONE for i, _ in infos)
            for (h, _, t, tol), d, j, (info, res) in zip(reqs, dev, ids, infos):
                ref, rres = alone(h, d, t, tol)
                assert bool((eng.output(j) == ref).all())
                assert same_result(res, rres)
            # the large-job lane keeps one job at a time, in submission order
            big = [infos[k][0] for k in (0, 2, 4)]
            assert big[0].finished <= big[1].admitted and big[1].finished <= big[2].admitted
            st = eng.stats()
            assert st.jobs_submitted == st.jobs_done == len(reqs) and st.jobs_running == 0
            assert st.pool_bytes <= budget
            with pytest.raises(te.TEError):
                eng.poll(len(reqs))


def test_engine_admission_by_footprint():
    te = lib()
    H, vs = W.xxz_chain(12, 41, n_v0=5)
    fp = te.te_job_footprint(4096, M)
    budget = int(2.5 * fp)
    with hamiltonian(H) as h:
        dev = [to_dev(v) for v in vs]
        with te.Engine(budget, m=M, max_jobs=16, **TUNE) as eng:
            announce("engine: 5 jobs, budget for 2")
            ids = [eng.submit(h, d, 10.0, 1e-8) for d in dev]
            eng.wait(-1, timeout=300)
            infos = [eng.poll(j)[0] for j in ids]
            assert all(i.state == te.TE_JOB_DONE for i in infos)
            # never more than two resident: at every admission at most one other job is resident
            for k, i in enumerate(infos):
                overlapping = sum(1 for q, o in enumerate(infos) if q != k and o.admitted <= i.admitted < o.finished)
                assert overlapping <= 1, k
            assert infos[2].admitted >= min(infos[0].finished, infos[1].finished)
            st = eng.stats()
            assert st.pool_peak <= 2 * fp + 4096
            for d, j in zip(dev, ids):
                ref, _ = alone(h, d, 10.0, 1e-8)
                assert bool((eng.output(j) == ref).all())
            # a job larger than the whole pool is refused at submission
            Hbig, vbig = W.xxz_chain(14, 42)
            with hamiltonian(Hbig) as hb:
                with pytest.raises(te.TEError) as ei:
                    eng.submit(hb, to_dev(vbig), 1.0, 1e-8)
                assert ei.value.status == te.TE_ERR_CAPACITY


def test_engine_edge_cases_do_not_disturb_the_mix():
    te = lib()
    H, vs = W.xxz_chain(10, 51, n_v0=2)
    import torch
    with hamiltonian(H) as h:
        good = to_dev(vs[0])
        zero = torch.zeros_like(good)
        bad = to_dev(vs[1])
        bad[7] = complex(float("nan"), 0.0)
        with te.Engine(8 * te.te_job_footprint(1024, M), m=M, max_jobs=8, threaded=False, **TUNE) as eng:
            announce("engine: t=0, zero v0, NaN v0 next to a normal job")
            j0 = eng.submit(h, good, 0.0, 1e-8)
            jz = eng.submit(h, zero, 5.0, 1e-8)
            jn = eng.submit(h, bad, 5.0, 1e-8)
            jg = eng.submit(h, good, 5.0, 1e-8)
            eng.wait(-1, timeout=120)
            i0, r0 = eng.poll(j0)
            assert i0.state == te.TE_JOB_DONE and r0.err_bound == 0 and bool((eng.output(j0) == good).all())
            iz, rz = eng.poll(jz)
            assert iz.state == te.TE_JOB_DONE and rz.err_bound == 0 and rz.t_reached == 5.0
            assert float(eng.output(jz).abs().max()) == 0.0
            inn, _ = eng.poll(jn)
            assert inn.state == te.TE_JOB_FAILED and inn.status == te.TE_ERR_NONFINITE
            ig, rg = eng.poll(jg)
            assert ig.state == te.TE_JOB_DONE
            ref, rref = alone(h, good, 5.0, 1e-8)
            assert bool((eng.output(jg) == ref).all()) and same_result(rg, rref)


def test_engine_profile_mode_accounts_every_kernel_class(mixed_groups):
    te = lib()
    H, vs, t, tol = mixed_groups[0]
    with hamiltonian(H) as h:
        d = [to_dev(v) for v in vs]
        announce("batch in profiling mode")
        outs_p, res_p, st = te.te_batch_run([(h, d, t, tol)], m=M, profile=True, **TUNE)
        outs_g, res_g, _ = te.te_batch_run([(h, d, t, tol)], m=M, **TUNE)
        for a, b in zip(outs_p[0], outs_g[0]):
            assert bool((a == b).all())
        prof = st.prof.as_dict()
        for k in te.KERNEL_CLASSES:
            assert prof[k]["launches"] > 0 and prof[k]["seconds"] > 0, k
        for k in ("project", "update", "combine"):
            assert prof[k]["bytes"] > 0, k
        rounds = max(r.steps for r, _, _ in res_p)
        assert prof["step"]["launches"] == rounds and st.rounds == rounds


def test_batch_sample_of_the_256_instance_workload():
    """Six instances of the 256-instance XXZ batch draw (L in 10..18, 1-8 vectors each)."""
    te = lib()
    jobs = W.batch_jobs()[:6]
    hs, groups, host = [], [], []
    for j in jobs:
        H, vs = j.build()
        h = hamiltonian(H)
        hs.append(h)
        host.append((H, vs))
        groups.append((h, [to_dev(v) for v in vs], j.t, j.tol))
    announce(f"batch sample: L={[j.L for j in jobs]} n_v0={[j.n_v0 for j in jobs]}")
    outs, results, stats = te.te_batch_run(groups, m=M, **TUNE)
    assert stats.jobs_done == sum(j.n_v0 for j in jobs)
    k = 0
    for gi, (h, d, t, tol) in enumerate(groups):
        for vi, v in enumerate(d):
            res, status, _ = results[k]
            k += 1
            assert status == te.TE_OK
            assert res.err_bound <= tol * (1 + 1e-12)
            assert abs(float(outs[gi][vi].norm()) - 1.0) <= 1e-9 + res.err_bound
            if vi == 0:
                announce(f"alone: instance {jobs[gi].index} L={jobs[gi].L}")
                ref, rres = alone(h, v, t, tol)
                assert bool((outs[gi][vi] == ref).all())
    for h in hs:
        h.destroy()
