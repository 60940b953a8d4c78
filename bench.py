#!/usr/bin/env python3
"""Throughput of the restarted Krylov evolution exp(-iHt) v0 on one MI355X.

One step = one complete te_evolve (every restart: sparse product + projections, basis
update, eigensolve + error integrals + step search, recombination) of the XXZ ring with
L=20 sites (d = 1,048,576, nnz = 11,534,336), t=100, tol=1e-8, m=40, on seeded synthetic
inputs already resident in device memory.  Prints ONE JSON line on stdout.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload xxz_L20]

The timed solves run in profiling mode (an event around every kernel), which yields the
per-kernel durations for the roofline entry; the same count of solves is also timed in the
default graph mode and reported as "graph_mode" (not the headline value).
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


def measured_traffic(kernel_source):
    """HBM bytes per projection launch from the committed counter runs, or None when the kernel
    source changed since they were taken (profiles/xxz_L20_hbm_traffic.json)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "xxz_L20_hbm_traffic.json")
    try:
        rec = json.load(open(path))
        src = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_arnoldi_hip") != src:
        return None
    return rec


def cpu_baseline(wl, gpu_restarts, n_restarts):
    """The CPU oracle, as it stands, on a bounded sample: its first n_restarts restarts of the same
    workload, extrapolated to a whole solve with the restart count of the GPU solve."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    t0 = time.perf_counter()
    res = oracle.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, max_steps=n_restarts)
    dt = time.perf_counter() - t0
    per_restart = dt / max(res.steps, 1)
    solve_s = per_restart * gpu_restarts
    return {
        "value": 1.0 / solve_s,
        "unit": "states/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"first {res.steps} restarts of {wl.name} ({dt:.1f} s, {per_restart:.2f} s/restart), "
                   f"extrapolated to the {gpu_restarts} restarts of one solve; sparse product single-threaded "
                   f"(SciPy), BLAS-1 on {threads} OpenBLAS threads"),
        "seconds_per_solve": solve_s,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="xxz_L20")
    ap.add_argument("--cpu-restarts", type=int, default=2, help="restarts of the CPU oracle sample (0: skip)")
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
    H = te.te_hamiltonian_create(wl.H.row_ptr, wl.H.col, wl.H.val)
    v0 = torch.from_numpy(wl.v0).to(dev)
    out = torch.empty_like(v0)
    plain = te.te_default_options()
    prof = te.te_default_options(flags=te.TE_OPT_PROFILE)

    for i in range(args.warmup):
        _, res = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=plain, out=out)
        log(f"[bench] warmup {i}: restarts={res.steps} bound={res.err_bound:.3e}")

    # ---- timed region (profiling mode: events around every kernel, on the call's stream)
    totals = {k: {"launches": 0, "seconds": 0.0, "bytes": 0.0} for k in te.KERNEL_CLASSES}
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s = time.perf_counter()
        _, res = te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=prof, out=out)
        lat.append(time.perf_counter() - s)
        p = te.te_last_profile(H).as_dict()
        for k in totals:
            for f in totals[k]:
                totals[k][f] += p[k][f]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    restarts, matvecs, bound = res.steps, res.matvecs, res.err_bound
    log(f"[bench] timed {args.steps} solves in {elapsed:.3f} s; restarts/solve={restarts}")

    # ---- same solves in graph mode (informational)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for i in range(args.steps):
        te.te_evolve(H, v0, wl.t, wl.tol, wl.m, options=plain, out=out)
    torch.cuda.synchronize()
    graph_elapsed = time.perf_counter() - g0

    kernel_gbs = {k: (v["bytes"] / v["seconds"] / 1e9 if v["seconds"] > 0 else None) for k, v in totals.items()}
    traffic = measured_traffic(os.path.join(ROOT, "paper_2205_15346_amd", "csrc", "arnoldi.hip"))
    dominant = max(totals, key=lambda k: totals[k]["seconds"])
    dom = totals[dominant]
    achieved = dom["bytes"] / dom["seconds"] / 1e9
    alg_bytes = sum(v["bytes"] for v in totals.values())
    kernel_seconds = sum(v["seconds"] for v in totals.values())

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
                   "seed": workloads.WORKLOADS[wl.name]["seed"]},
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic["project_bytes_per_launch"] if (traffic and dominant == "project") else None,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": dom["bytes"] / max(dom["launches"], 1),
        },
        "cpu_baseline": {k: v for k, v in cpu.items() if k != "seconds_per_solve"} if cpu else None,
        "hbm_gbs_algorithmic_all_kernels": alg_bytes / kernel_seconds / 1e9,
        "hbm_gbs_algorithmic_wall": alg_bytes / elapsed / 1e9,
        "kernel_gbs": kernel_gbs,
        "kernel_ms_per_solve": {k: 1e3 * v["seconds"] / args.steps for k, v in totals.items()},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "restarts_per_solve": restarts,
        "matvecs_per_solve": matvecs,
        "err_bound": bound,
        "graph_mode": {"ms_per_step": 1e3 * graph_elapsed / args.steps, "value": args.steps / graph_elapsed},
    }
    H.destroy()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
