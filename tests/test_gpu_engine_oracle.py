"""Batched and served results against the CPU oracle on seeded samples of at least 16 jobs of
the batch and serving draws.  The samples keep the draws' structure (t, tol, one Hamiltonian per
instance or per (kind, size), several vectors per instance) at sizes the oracle finishes in
seconds: batch instances with L <= 12; serving requests with XXZ L in 12..14 and Bose K = N in
7..8 (the full-size draws run in bench.py).  Bar: ||v_gpu - v_oracle|| <= 2 tol + 1e-12."""

import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host

pytestmark = pytest.mark.gpu
M = 40


def test_batch_draw_sample_matches_oracle():
    te = lib()
    picked, n = [], 0
    for job in W.batch_jobs():
        if job.L <= 12:
            picked.append(job)
            n += job.n_v0
        if n >= 16:
            break
    assert n >= 16
    hs, groups, host = [], [], []
    for job in picked:
        H, vs = job.build()
        h = hamiltonian(H)
        hs.append(h)
        host.append((H, vs, job))
        groups.append((h, [to_dev(v) for v in vs], job.t, job.tol))
    announce(f"batch sample vs oracle: {len(picked)} instances, {n} jobs")
    outs, results, stats = te.te_batch_run(groups, m=M)
    k = 0
    for gi, (H, vs, job) in enumerate(host):
        for vi, v in enumerate(vs):
            res, status, _ = results[k]
            k += 1
            assert status == te.TE_OK
            ro = O.evolve(H, v, job.t, job.tol, M)
            diff = np.linalg.norm(to_host(outs[gi][vi]) - ro.v)
            assert diff <= 2 * job.tol + 1e-12, (job.index, vi, diff)
    for h in hs:
        h.destroy()


def test_serving_draw_sample_matches_oracle():
    te = lib()
    reqs = W.serving_requests(16, 8.0, xxz_sizes=(12, 15), bose_sizes=(7, 9))
    mats, hs = {}, {}
    for r in reqs:
        key = r.hamiltonian_key()
        if key not in mats:
            mats[key] = W.configs.serving_hamiltonian(*key)
            hs[key] = hamiltonian(mats[key])
    v0 = [r.v0(mats[r.hamiltonian_key()].dim) for r in reqs]
    budget = 4 * max(te.te_job_footprint(m.dim, M) for m in mats.values())
    announce(f"serving sample vs oracle: {len(reqs)} requests, {len(mats)} Hamiltonians")
    with te.Engine(budget, m=M, max_jobs=8) as eng:
        ids = []
        t0 = time.perf_counter()
        for r, v in zip(reqs, v0):
            delay = r.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(eng.submit(hs[r.hamiltonian_key()], to_dev(v), r.t, r.tol))
        eng.wait(-1, timeout=300)
        got = [(eng.poll(j), to_host(eng.output(j))) for j in ids]
        assert eng.stats().pool_peak <= budget
    for r, v, ((info, res), out) in zip(reqs, v0, got):
        assert info.state == te.TE_JOB_DONE
        ro = O.evolve(mats[r.hamiltonian_key()], v, r.t, r.tol, M)
        diff = np.linalg.norm(out - ro.v)
        assert diff <= 2 * r.tol + 1e-12, (r.index, r.kind, r.size, diff)
    for h in hs.values():
        h.destroy()
