#!/usr/bin/env python3
"""Throughput of the restarted Krylov evolution exp(-iHt) v0 on one MI355X.

One step = one complete te_evolve (every restart: sparse product + projections, basis
update, eigensolve + error integrals + step search, recombination) of the XXZ ring with
L=20 sites (d = 1,048,576, nnz = 11,534,336), t=100, tol=1e-8, m=40, on seeded synthetic
inputs already resident in device memory.  Prints ONE JSON line on stdout.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload xxz_L20]

The timed solves run in profiling mode (an event around every kernel), which yields the
per-kernel durations for the roofline entry; the same count of solves is also timed in the
default graph mode and reported as "graph_mode" (not the headline value).  The same line
carries informational entries: the three-term mode, the solve with the matrix kept as complex
CSR ("csr_storage", with its own roofline), the Bose chain K = N = 12 at m = 60 ("bose_K12"),
the paper's own example ("paper_model"), the 256-instance batch against the same jobs one at a
time ("batch"), serving with Poisson arrivals at 70% of the measured saturation against a FIFO
server of single solves ("serving"), and the CPU oracle on a bounded sample ("cpu_baseline").
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Krylov exp(-iHt)v: HBM GB/s, evolved states/sec at tol 1e-8, p50/p99"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def measured_traffic(kernel_source, record="xxz_L20_hbm_traffic.json"):
    """HBM bytes per projection launch from a committed counter record under profiles/, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    try:
        rec = json.load(open(path))
        src = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_arnoldi_hip") != src:
        return None
    return rec


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, gpu_restarts, n_restarts, single_thread_restarts=1):
    """The CPU oracle, as it stands, on a bounded sample: its first n_restarts restarts of the same
    workload on the host's BLAS threads, and single_thread_restarts more with BLAS limited to one
    thread, each extrapolated to a whole solve with the restart count of the GPU solve."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    t0 = time.perf_counter()
    res = oracle.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, max_steps=n_restarts)
    dt = time.perf_counter() - t0
    per_restart = dt / max(res.steps, 1)
    solve_s = per_restart * gpu_restarts
    rec = {
        "value": 1.0 / solve_s,
        "unit": "states/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"first {res.steps} restarts of {wl.name} ({dt:.1f} s, {per_restart:.2f} s/restart), "
                   f"extrapolated to the {gpu_restarts} restarts of one solve; sparse product single-threaded "
                   f"(SciPy), BLAS-1 on {threads} OpenBLAS threads"),
        "cpu_model": cpu_model(),
        "seconds_per_solve": solve_s,
    }
    if single_thread_restarts > 0:
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            r1 = oracle.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, max_steps=single_thread_restarts)
            d1 = time.perf_counter() - t1
        p1 = d1 / max(r1.steps, 1)
        rec["single_thread"] = {"value": 1.0 / (p1 * gpu_restarts), "unit": "states/s", "cores": 1,
                                "sample": f"first {r1.steps} restart(s), {p1:.2f} s/restart, BLAS on one thread"}
    return rec


def kernel_rates(prof):
    return {k: (v["bytes"] / v["seconds"] / 1e9 if v["seconds"] > 0 and v["bytes"] > 0 else None)
            for k, v in prof.items()}


def time_solves(te, torch, H, v0, out, wl, steps, warmup, label):
    """warmup untimed solves, then `steps` solves in profiling mode (HIP events bound to every
    kernel dispatch, on the call's stream); per-kernel totals, wall time, latencies, last result."""
    plain = te.te_default_options()
    prof = te.te_default_options(flags=te.TE_OPT_PROFILE)
    for i in range(warmup):
        _, res = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=plain, out=out)
        log(f"[bench] {label} warmup {i}: restarts={res.steps} bound={res.err_bound:.3e}")
    totals = {k: {"launches": 0, "seconds": 0.0, "bytes": 0.0} for k in te.KERNEL_CLASSES}
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        s = time.perf_counter()
        _, res = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=prof, out=out)
        lat.append(time.perf_counter() - s)
        p = te.te_last_profile(H).as_dict()
        for k in totals:
            for f in totals[k]:
                totals[k][f] += p[k][f]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] {label}: {steps} solves in {elapsed:.3f} s; restarts/solve={res.steps} bound={res.err_bound:.3e}")
    return {"totals": totals, "elapsed": elapsed, "lat": lat, "res": res}


def roofline_of(totals, traffic=None):
    """Roofline entry of the dominant kernel class: its algorithmic bytes over the summed
    durations of its launches (HIP events on the call's stream)."""
    dominant = max(totals, key=lambda k: totals[k]["seconds"])
    dom = totals[dominant]
    achieved = dom["bytes"] / dom["seconds"] / 1e9
    return {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": dom["bytes"] / max(dom["launches"], 1)}


def survey_bytes_per_restart(d, nnz, m):
    """Algorithmic bytes of one restart's Krylov build with full Gram-Schmidt and the matrix as
    complex CSR (20 bytes per entry): iteration j = 1..m moves 20 nnz + 4 (d + 1) + 16 d (2j + 5)."""
    return sum(20.0 * nnz + 4.0 * (d + 1) + 16.0 * d * (2 * j + 5) for j in range(1, m + 1))


def spmv_orth_rates(totals, d, nnz, m, restarts_total):
    """Sparse product + orthogonalisation (projection, fold and update kernels together): the
    library's own algorithmic bytes and the complex-CSR bytes of the formula above, each over the
    same kernel time."""
    ks = ("project", "fold", "update")
    sec = sum(totals[k]["seconds"] for k in ks)
    own = sum(totals[k]["bytes"] for k in ks) / sec / 1e9
    csr = survey_bytes_per_restart(d, nnz, m) * restarts_total / sec / 1e9
    return {"kernels": list(ks), "gbs": own, "frac_of_peak": own / HBM_PEAK_GBS,
            "gbs_on_complex_csr_bytes": csr, "frac_on_complex_csr_bytes": csr / HBM_PEAK_GBS}


def bench_workload(te, torch, dev, name, steps, warmup, shape="auto", store_csr=False):
    """One single-solve configuration other than the headline, timed like the headline."""
    import workloads
    wl = workloads.workload(name)
    H = te.te_hamiltonian_create(wl.H.row_ptr, wl.H.col, wl.H.val, store_csr=store_csr)
    v0 = torch.from_numpy(wl.v0).to(dev)
    out = torch.empty_like(v0)
    if shape != "auto":
        te.te_set_tuning(H, *shape)
    r = time_solves(te, torch, H, v0, out, wl, steps, warmup, name)
    res = r["res"]
    tuning = te.te_get_tuning(H).as_dict()
    roof = roofline_of(r["totals"])
    traffic = measured_traffic(os.path.join(ROOT, "paper_2205_15346_amd", "csrc", "arnoldi.hip"),
                               f"{name}_{'csr_' if store_csr else ''}hbm_traffic.json")
    shape_now = [tuning[k] for k in ("lanes_per_row", "nnz_per_lane", "rows_per_thread", "update_rows_per_thread",
                                     "split_projection")]
    if traffic and traffic.get("shape") == shape_now and roof["kernel"] == "project":
        roof["traffic"] = traffic["project_bytes_per_launch"]
    rec = {"workload": name, "dim": wl.H.dim, "nnz": wl.H.nnz, "t": wl.t, "tol": wl.tol, "m": wl.m,
           "storage": H.storage, "kernel_shape": tuning,
           "value": steps / r["elapsed"], "unit": "states/s", "ms_per_step": 1e3 * r["elapsed"] / steps,
           "restarts_per_solve": res.steps, "matvecs_per_solve": res.matvecs, "err_bound": res.err_bound,
           "warnings": res.warnings, "roofline": roof,
           "spmv_orthogonalisation": spmv_orth_rates(r["totals"], wl.H.dim, wl.H.nnz, wl.m, res.steps * steps),
           "kernel_ms_per_solve": {k: 1e3 * v["seconds"] / steps for k, v in r["totals"].items()}}
    H.destroy()
    return rec


def bench_three_term(te, torch, H, v0, out, wl, steps):
    """The headline solve with TE_OPT_LANCZOS3 (three-term recurrence, no re-orthogonalisation)."""
    o3 = te.te_default_options(flags=te.TE_OPT_PROFILE | te.TE_OPT_LANCZOS3)
    te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=o3, out=out)
    t3 = {k: {"seconds": 0.0, "bytes": 0.0} for k in te.KERNEL_CLASSES}
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for i in range(steps):
        _, res3 = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=o3, out=out)
        p = te.te_last_profile(H).as_dict()
        for k in t3:
            t3[k]["seconds"] += p[k]["seconds"]
            t3[k]["bytes"] += p[k]["bytes"]
    torch.cuda.synchronize()
    e3 = time.perf_counter() - s0
    log(f"[bench] three-term mode: {1e3 * e3 / steps:.1f} ms per solve, restarts={res3.steps}, "
        f"bound={res3.err_bound:.3e}")
    return {
        "value": steps / e3, "ms_per_step": 1e3 * e3 / steps, "restarts_per_solve": res3.steps,
        "err_bound": res3.err_bound,
        "kernel_gbs": {k: (v["bytes"] / v["seconds"] / 1e9 if v["seconds"] > 0 and v["bytes"] > 0 else None)
                       for k, v in t3.items()},
        "kernel_ms_per_solve": {k: 1e3 * v["seconds"] / steps for k, v in t3.items()},
    }


def bench_batch(te, torch, dev, n_instances, m, profile, reference=True):
    """The 256-instance XXZ batch (L ~ U{10..18}, 1-8 vectors each, t ~ U[1,100], tol in
    {1e-6, 1e-8, 1e-10}) through te_batch_*, against the same jobs one at a time through
    te_evolve.  Latency of a job = time from the start of the run to its result."""
    import workloads
    jobs = workloads.batch_jobs(n_instances)
    groups = []
    b0 = time.perf_counter()
    for j in jobs:
        H, vs = j.build()
        h = te.te_hamiltonian_create(H.row_ptr, H.col, H.val)
        groups.append((h, [torch.from_numpy(v).to(dev) for v in vs], j.t, j.tol))
    n_jobs = sum(len(g[1]) for g in groups)
    rows = sum(g[0].dim * len(g[1]) for g in groups)
    log(f"[bench] batch: {len(groups)} Hamiltonians, {n_jobs} jobs, {rows / 1e6:.1f}M rows "
        f"(built in {time.perf_counter() - b0:.1f} s)")
    te.te_batch_run(groups[:4], m=m)  # warm-up: load the batched kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, results, stats = te.te_batch_run(groups, m=m)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    lat = [info.finished - info.submitted for _, _, info in results]
    failed = sum(1 for _, s, _ in results if s != te.TE_OK)
    log(f"[bench] batch: {batch_s:.2f} s, {n_jobs / batch_s:.1f} states/s, rounds={stats.rounds} "
        f"plans={stats.plans} shape={stats.tuning.lanes_per_row}x{stats.tuning.nnz_per_lane}")
    prof = None
    if profile:
        _, _, pst = te.te_batch_run(groups, m=m, shape=(stats.tuning.lanes_per_row, stats.tuning.nnz_per_lane),
                                    profile=True)
        prof = pst.prof.as_dict()
    # one at a time through te_evolve (each handle autotunes its own shape on first use)
    seq_done = []
    worst = 0.0
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    k = 0
    for gi, (h, vs, t, tol) in enumerate(groups if reference else []):
        for vi, v in enumerate(vs):
            out, res = te.te_evolve(h, v, t, tol, m)
            seq_done.append(time.perf_counter() - s0)
            # two valid results differ by at most the two bounds plus the rounding of the two
            # computations (the paper's roundoff estimate), since the shapes differ
            allowed = (res.err_bound + results[k][0].err_bound + res.num_err_estimate
                       + results[k][0].num_err_estimate)
            worst = max(worst, float((out - outs[gi][vi]).norm()) / max(allowed, 1e-300))
            k += 1
    seq_s = time.perf_counter() - s0
    if reference:
        log(f"[bench] one at a time: {seq_s:.2f} s, {n_jobs / seq_s:.1f} states/s")

    for g in groups:
        g[0].destroy()
    rec = {
        "workload": f"xxz_batch_{n_instances}",
        "instances": len(groups), "jobs": n_jobs, "rows": rows, "m": m,
        "states_per_s": n_jobs / batch_s, "seconds": batch_s,
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "one_at_a_time": {"states_per_s": n_jobs / seq_s, "seconds": seq_s,
                          "latency_ms": {"p50": 1e3 * percentile(seq_done, 50), "p99": 1e3 * percentile(seq_done, 99)}}
        if reference else None,
        "speedup_vs_one_at_a_time": seq_s / batch_s if reference else None,
        "rounds": stats.rounds, "plans": stats.plans, "failed": failed,
        "pool_peak_gb": stats.pool_peak / 1e9,
        "shape": {"lanes_per_row": stats.tuning.lanes_per_row, "nnz_per_lane": stats.tuning.nnz_per_lane,
                  "update_rows_per_thread": stats.tuning.update_rows_per_thread},
        "max_diff_over_bounds_and_roundoff_vs_one_at_a_time": worst if reference else None,
    }
    if prof:
        rec["profile"] = {"kernel_gbs": kernel_rates(prof),
                          "kernel_s": {k: v["seconds"] for k, v in prof.items()},
                          "alg_gbs_all_kernels": sum(v["bytes"] for v in prof.values())
                          / max(sum(v["seconds"] for v in prof.values()), 1e-12) / 1e9}
    return rec


def serve_engine(te, torch, hs, reqs, v0, m, budget_gb, arrivals, label, lane_rows=0, lane_jobs=0):
    """Submit reqs at the given arrival times (seconds from the start) into a threaded engine;
    returns per-request (submitted, finished, info, result) and the engine stats."""
    small = min(hs.values(), key=lambda h: h.dim)
    vw = torch.zeros(small.dim, dtype=torch.complex128, device=v0[0].device)
    vw[0] = 1.0
    with te.Engine(int(budget_gb * 1e9), m=m, max_jobs=256, lane_rows=lane_rows, lane_jobs=lane_jobs) as eng:
        w = eng.submit(small, vw, 1.0, 1e-8)  # warm-up (kernels, tuning)
        eng.wait(w, timeout=600)
        torch.cuda.synchronize()
        ids = []
        t0 = time.perf_counter()
        for i, (r, v, at) in enumerate(zip(reqs, v0, arrivals)):
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(eng.submit(hs[r.hamiltonian_key()], v, r.t, r.tol))
            if (i + 1) % 25 == 0:
                log(f"[bench] {label}: {i + 1} requests submitted")
        while True:
            try:
                eng.wait(-1, timeout=30.0)
                break
            except te.TEError as e:
                if e.status != te.TE_ERR_TIMEOUT:
                    raise
                st = eng.stats()
                log(f"[bench] {label}: {st.jobs_done} done, {st.jobs_running} running, {st.jobs_queued} queued")
        infos = [eng.poll(j) for j in ids]
        outs = [eng.output(j).clone() for j in ids]
        st = eng.stats()
    return infos, outs, st


def latency_summary(lat):
    return {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)}


def bench_serving(te, torch, dev, n_requests, qps, m, budget_gb, sweep=(), sweep_requests=48,
                  saturation=False, saturation_requests=0, lane_rows=0, lane_jobs=0):
    """Poisson arrivals of XXZ (L 14..22) and Bose (K=N 10..12) requests into the threaded engine
    (continuous batching, admission by footprint), against the same stream served one request at a
    time by te_evolve (FIFO: completion = max(arrival, previous completion) + measured solve time).
    The draws of kind, size, t and tol do not depend on the QPS (only the gaps scale), so one set
    of one-at-a-time solve times serves every QPS.  saturation: all requests at time 0 first, and
    qps <= 0 then means 70% of the saturation throughput."""
    import workloads
    n_max = max([n_requests] + ([sweep_requests] if sweep else []))
    base = workloads.serving_requests(n_max, 1.0)  # arrivals at 1 QPS; scaled below
    hs = {}
    b0 = time.perf_counter()
    for r in base:
        key = r.hamiltonian_key()
        if key not in hs:
            H = workloads.configs.serving_hamiltonian(*key)
            hs[key] = te.te_hamiltonian_create(H.row_ptr, H.col, H.val)
            del H
    v0 = [torch.from_numpy(r.v0(hs[r.hamiltonian_key()].dim)).to(dev) for r in base]
    log(f"[bench] serving: up to {n_max} requests over {len(hs)} Hamiltonians (built in {time.perf_counter() - b0:.1f} s)")

    # one request at a time through te_evolve: service times (also the reference results)
    small = min(hs.values(), key=lambda h: h.dim)
    vw = torch.zeros(small.dim, dtype=torch.complex128, device=dev)
    vw[0] = 1.0
    te.te_evolve(small, vw, 1.0, 1e-8, m)
    service, ref = [], []
    for i, (r, v) in enumerate(zip(base, v0)):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        out, rr = te.te_evolve(hs[r.hamiltonian_key()], v, r.t, r.tol, m)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - s0)
        ref.append((out.clone(), rr.err_bound + rr.num_err_estimate))
        if (i + 1) % 25 == 0:
            log(f"[bench] one at a time: {i + 1} requests")

    def fifo(arrivals, n):
        done, lat = 0.0, []
        for at, sv in zip(arrivals[:n], service[:n]):
            done = max(done, at) + sv
            lat.append(done - at)
        return n / (done - arrivals[0]), lat

    def run(n, q, label):
        reqs = base[:n]
        arrivals = [0.0] * n if q is None else [r.arrival / q for r in reqs]
        infos, outs, st = serve_engine(te, torch, hs, reqs, v0[:n], m, budget_gb, arrivals, label, lane_rows,
                                       lane_jobs)
        first = min(i.submitted for i, _ in infos)
        last = max(i.finished for i, _ in infos)
        lat = [i.finished - i.submitted for i, _ in infos]
        worst = max(float((o - ref[k][0]).norm())
                    / max(ref[k][1] + infos[k][1].err_bound + infos[k][1].num_err_estimate, 1e-300)
                    for k, o in enumerate(outs))
        f_rate, f_lat = fifo(arrivals, n)
        rec = {"requests": n, "qps": q, "states_per_s": n / (last - first), "seconds": last - first,
               "latency_ms": latency_summary(lat),
               "one_at_a_time_fifo": {"states_per_s": f_rate, "latency_ms": latency_summary(f_lat)},
               "rounds": st.rounds, "plans": st.plans, "pool_peak_gb": st.pool_peak / 1e9,
               "failed": sum(1 for i, _ in infos if i.state != te.TE_JOB_DONE),
               "max_diff_over_bounds_and_roundoff_vs_one_at_a_time": worst,
               # the requests behind the tail: the three slowest in the engine
               "slowest": [{"request": k, "kind": reqs[k].kind, "size": reqs[k].size, "t": reqs[k].t,
                            "tol": reqs[k].tol, "latency_s": lat[k], "fifo_latency_s": f_lat[k],
                            "solve_alone_s": service[k]}
                           for k in sorted(range(n), key=lambda k: -lat[k])[:3]]}
        log(f"[bench] {label}: {rec['states_per_s']:.2f} states/s, p50 {rec['latency_ms']['p50'] / 1e3:.3f} s, "
            f"p99 {rec['latency_ms']['p99'] / 1e3:.3f} s | one at a time {f_rate:.2f} states/s, "
            f"p50 {rec['one_at_a_time_fifo']['latency_ms']['p50'] / 1e3:.3f} s, "
            f"p99 {rec['one_at_a_time_fifo']['latency_ms']['p99'] / 1e3:.3f} s")
        return rec

    out = {"m": m, "hbm_budget_gb": budget_gb, "lane_rows": lane_rows, "lane_jobs": lane_jobs,
           "mean_service_ms": 1e3 * sum(service[:n_requests]) / n_requests,
           "one_at_a_time_saturation_states_per_s": n_requests / sum(service[:n_requests])}
    if saturation:
        n_sat = saturation_requests or n_requests
        sat = run(n_sat, None, f"saturation ({n_sat} requests at t=0)")
        out["saturation"] = sat
        if qps <= 0:
            qps = 0.7 * sat["states_per_s"]
    main = run(n_requests, qps, f"serving {n_requests} at {qps:.2f} qps")
    out.update({"workload": f"serving_{n_requests}_at_{qps:.2f}qps", **main})
    if sweep:
        out["sweep"] = [run(sweep_requests, q, f"sweep {sweep_requests} at {q} qps") for q in sweep]
    for h in hs.values():
        h.destroy()
    return out


def bench_paper_model(te, torch, dev, packed_only=False):
    """The paper's own performance example (Sec. "Analysis of Performance"): eq. fullHamiltonianSimple
    with K = K' = 10, N_m = 5, N_0 = N_c = 100 (d = 1,565,904), the initial state of eq.
    initialStateSimple, t = 10, m = 40, err_max = 1e-7.  The paper's figure (one CPU thread of an
    i9-9900K, 353 s; roundoff estimate 3.2e-6) is context, not a comparison on equal hardware."""
    import workloads
    params = dict(K=10, Kp=10, Nm=5, N0=100, Nc=100.0)
    host_build_s = None
    if not packed_only:
        b0 = time.perf_counter()
        H, _, _ = workloads.memory_burden_model(**params)  # host builder: basis, lookup, triplets
        host_build_s = time.perf_counter() - b0
        del H
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    h, idx = te.te_hamiltonian_create_memory_burden(**params)  # the same matrix built on the device
    torch.cuda.synchronize()
    build_s = time.perf_counter() - b0
    x = torch.zeros(h.dim, dtype=torch.complex128, device=dev)
    x[idx] = 1.0  # eq. initialStateSimple
    dim, nnz = h.dim, h.nnz
    log(f"[bench] paper model built on the device in {build_s:.3f} s (host builder: {host_build_s} s)")
    def timed():
        te.te_evolve(h, x, 10.0, 1e-7, 40)  # warm-up and autotune
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            out, res = te.te_evolve(h, x, 10.0, 1e-7, 40)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - s0)
        return sum(times) / len(times), out, res

    storage_built = h.storage
    if packed_only:
        sec_csr, out_csr, res_csr = None, None, None
    else:
        sec_csr, out_csr, res_csr = timed()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    storage = te.te_hamiltonian_pack(h)  # value codes: the couplings take a few hundred values
    pack_s = time.perf_counter() - p0
    sec, out, res = timed()
    h.destroy()
    agree = None if packed_only else float((out - out_csr).norm()) / (
        res.err_bound + res_csr.err_bound + res.num_err_estimate + res_csr.num_err_estimate)
    unpacked = "" if packed_only else f"{sec_csr:.3f} s as {storage_built} entries, "
    log(f"[bench] paper model d={dim}: {sec:.3f} s per solve ({storage}; {unpacked}packed in {pack_s:.2f} s), "
        f"restarts={res.steps}, bound={res.err_bound:.2e}, roundoff estimate={res.num_err_estimate:.2e}")
    return {"dim": dim, "nnz": nnz, "t": 10.0, "tol": 1e-7, "m": 40, "seconds_per_solve": sec, "storage": storage,
            "seconds_per_solve_unpacked": sec_csr, "storage_unpacked": storage_built, "pack_seconds": pack_s,
            "diff_packed_vs_unpacked_over_bounds_and_roundoff": agree,
            "restarts": res.steps, "err_bound": res.err_bound, "num_err_estimate": res.num_err_estimate,
            "warnings": res.warnings, "build_seconds_device": build_s, "build_seconds_host_builder": host_build_s,
            "paper_context": {"seconds_one_cpu_thread_i9_9900K": 353.0, "num_err_estimate": 3.2e-6}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="xxz_L20")
    ap.add_argument("--cpu-restarts", type=int, default=2, help="restarts of the CPU oracle sample (0: skip)")
    ap.add_argument("--shape", default="1,8,4,2,0",
                    help="projection kernel shape lanes,nnz,rows,update_rows,split for the single solve "
                         "(default: the shape te_autotune selects for this matrix on MI355X), or 'auto'")
    ap.add_argument("--storage", choices=["packed", "csr"], default="packed",
                    help="matrix storage of the timed solves: packed entries where the matrix allows "
                         "(default), or the CSR as given")
    ap.add_argument("--three-term", type=int, default=1, help="also time the three-term mode (0: skip)")
    ap.add_argument("--csr-storage", type=int, default=1,
                    help="also time the solve with the matrix kept as CSR instead of packed (0: skip)")
    ap.add_argument("--batch-instances", type=int, default=256, help="instances of the XXZ batch (0: skip)")
    ap.add_argument("--batch-profile", type=int, default=1, help="also run the batch in profiling mode")
    ap.add_argument("--batch-reference", type=int, default=1,
                    help="also run the batch's jobs one at a time (0: skip; for kernel profiles of the batch)")
    ap.add_argument("--serve-requests", type=int, default=120, help="requests of the serving run (0: skip)")
    ap.add_argument("--serve-qps", type=float, default=0.0, help="arrival rate; <= 0: 70%% of the saturation rate")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0)
    ap.add_argument("--serve-saturation", type=int, default=0, help="first measure saturation (all arrive at 0)")
    ap.add_argument("--serve-saturation-requests", type=int, default=60,
                    help="requests of the saturation run (0: as many as the serving run)")
    ap.add_argument("--serve-lane-rows", type=int, default=1 << 20,
                    help="engine lanes: jobs of at least this many rows in a lane of their own (0: one lane)")
    ap.add_argument("--serve-lane-jobs", type=int, default=3,
                    help="resident jobs of the large-job lane (3: the lowest p99 at the default operating point)")
    ap.add_argument("--serve-sweep", default="", help="comma-separated QPS values for a sweep")
    ap.add_argument("--serve-sweep-requests", type=int, default=48)
    ap.add_argument("--paper-model", type=int, default=2,
                    help="also time the paper's own performance example (d = 1,565,904), built on the device: "
                         "1 = as built (real CSR) and packed, plus the host builder's time; 2 = packed only; "
                         "0 = skip")
    ap.add_argument("--bose-solves", type=int, default=2,
                    help="timed solves of the Bose chain K = N = 12 (d = 1,352,078, t = 50, tol = 1e-10, "
                         "m = 60; 0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path (independent solves shard "
            "without communication; see DESIGN.md).  Run with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2205_15346_amd import te

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = workloads.workload(args.workload)
    log(f"[bench] workload {wl.name}: d={wl.H.dim} nnz={wl.H.nnz} t={wl.t} tol={wl.tol} m={wl.m}")
    H = te.te_hamiltonian_create(wl.H.row_ptr, wl.H.col, wl.H.val, store_csr=args.storage == "csr")
    v0 = torch.from_numpy(wl.v0).to(dev)
    out = torch.empty_like(v0)
    plain = te.te_default_options()

    if args.shape != "auto":
        te.te_set_tuning(H, *[int(x) for x in args.shape.split(",")])
    if args.warmup > 0:
        _, res = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=plain, out=out)  # autotunes when asked
    tuning = te.te_get_tuning(H).as_dict()
    log(f"[bench] kernel shape: {tuning}")

    # ---- timed region (profiling mode: events around every kernel, on the call's stream)
    head = time_solves(te, torch, H, v0, out, wl, args.steps, max(args.warmup - 1, 0), wl.name)
    totals, elapsed, lat, res = head["totals"], head["elapsed"], head["lat"], head["res"]
    restarts, matvecs, bound = res.steps, res.matvecs, res.err_bound

    # ---- same solves in graph mode (informational)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for i in range(args.steps):
        te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=plain, out=out)
    torch.cuda.synchronize()
    graph_elapsed = time.perf_counter() - g0

    # ---- three-term mode (TE_OPT_LANCZOS3; informational, not the headline)
    three_term = bench_three_term(te, torch, H, v0, out, wl, args.steps) if args.three_term else None

    # ---- the same workload with the matrix kept as complex CSR (TE_STORE_CSR), in the shape the
    # autotuner picks for it, timed the same way (informational)
    csr = None
    if args.csr_storage:
        csr = bench_workload(te, torch, dev, wl.name, min(args.steps, 5), 1, shape=(8, 2, 4, 2, 1),
                             store_csr=True)
        csr_traffic = measured_traffic(os.path.join(ROOT, "paper_2205_15346_amd", "csrc", "arnoldi.hip"),
                                       "xxz_L20_csr_hbm_traffic.json")
        if csr_traffic and csr_traffic.get("shape") == [8, 2, 4, 2, 1] and csr["roofline"]["kernel"] == "project":
            csr["roofline"]["traffic"] = csr_traffic["project_bytes_per_launch"]
        log(f"[bench] CSR storage ({csr['storage']}): {csr['ms_per_step']:.1f} ms per solve, "
            f"{csr['roofline']['kernel']} at {csr['roofline']['achieved']:.0f} GB/s")

    kernel_gbs = {k: (v["bytes"] / v["seconds"] / 1e9 if v["seconds"] > 0 else None) for k, v in totals.items()}
    traffic = measured_traffic(os.path.join(ROOT, "paper_2205_15346_amd", "csrc", "arnoldi.hip"),
                               f"{wl.name}_{'csr_' if args.storage == 'csr' else ''}hbm_traffic.json")
    shape = [tuning[k] for k in ("lanes_per_row", "nnz_per_lane", "rows_per_thread", "update_rows_per_thread",
                                 "split_projection")]
    if traffic and traffic.get("shape") != shape:
        traffic = None  # the counters were taken on another kernel shape
    roof = roofline_of(totals)
    if traffic and roof["kernel"] == "project":
        roof["traffic"] = traffic["project_bytes_per_launch"]
    roof["storage"] = H.storage
    alg_bytes = sum(v["bytes"] for v in totals.values())
    kernel_seconds = sum(v["seconds"] for v in totals.values())

    H.destroy()
    batch = serving = None
    if args.batch_instances > 0:
        batch = bench_batch(te, torch, dev, args.batch_instances, wl.m, bool(args.batch_profile),
                            bool(args.batch_reference))
    if args.serve_requests > 0:
        sweep = [float(x) for x in args.serve_sweep.split(",") if x.strip()]
        serving = bench_serving(te, torch, dev, args.serve_requests, args.serve_qps, wl.m, args.serve_budget_gb,
                                sweep, args.serve_sweep_requests, bool(args.serve_saturation) or args.serve_qps <= 0,
                                args.serve_saturation_requests, args.serve_lane_rows, args.serve_lane_jobs)
    paper = bench_paper_model(te, torch, dev, packed_only=args.paper_model == 2) if args.paper_model else None
    bose = None
    if args.bose_solves > 0:
        # the shape the autotuner picks on this matrix in most runs (its neighbours are within 2%),
        # pinned so that every run times the same kernels and the counter record applies
        bose = bench_workload(te, torch, dev, "bose_K12", args.bose_solves, 1, shape=(2, 8, 4, 1, 1))
        log(f"[bench] bose_K12: {bose['ms_per_step']:.1f} ms per solve, {bose['restarts_per_solve']} restarts, "
            f"{bose['roofline']['kernel']} at {bose['roofline']['achieved']:.0f} GB/s ({bose['storage']})")

    cpu = None
    if args.cpu_restarts > 0:
        log(f"[bench] CPU oracle sample: {args.cpu_restarts} restarts")
        cpu = cpu_baseline(wl, restarts, args.cpu_restarts)
        log(f"[bench] CPU oracle: {cpu['seconds_per_solve']:.1f} s per solve")

    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "dim": wl.H.dim, "nnz": wl.H.nnz, "t": wl.t, "tol": wl.tol, "m": wl.m,
                   "storage": H.storage,
                   "seed": workloads.WORKLOADS[wl.name]["seed"]},
        "roofline": roof,
        "cpu_baseline": {k: v for k, v in cpu.items() if k != "seconds_per_solve"} if cpu else None,
        "hbm_gbs_algorithmic_all_kernels": alg_bytes / kernel_seconds / 1e9,
        "spmv_orthogonalisation": spmv_orth_rates(totals, wl.H.dim, wl.H.nnz, wl.m, restarts * args.steps),
        "hbm_gbs_algorithmic_wall": alg_bytes / elapsed / 1e9,
        "kernel_gbs": kernel_gbs,
        "kernel_ms_per_solve": {k: 1e3 * v["seconds"] / args.steps for k, v in totals.items()},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "restarts_per_solve": restarts,
        "matvecs_per_solve": matvecs,
        "err_bound": bound,
        "graph_mode": {"ms_per_step": 1e3 * graph_elapsed / args.steps, "value": args.steps / graph_elapsed},
        "csr_storage": csr,
        "kernel_shape": tuning,
        "three_term_mode": three_term,
        "batch": batch,
        "serving": serving,
        "paper_model": paper,
        "bose_K12": bose,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
