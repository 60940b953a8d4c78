"""Write the oracle's final states for the full-size single-solve workloads.

    python tests/golden/make_oracle_states.py xxz_L20 [bose_K12 ...]

For each named workload (``workloads.WORKLOADS``) this builds the seeded Hamiltonian and
initial vector, runs ``oracle.evolve`` (Alg. 1 of the paper, plain NumPy/SciPy FP64) to the
workload's time, and stores

  oracle_state_<name>.npy    v(t), complex128, the oracle's result
  oracle_state_<name>.json   the oracle's step count, matrix-vector products, bound, roundoff
                             estimate, warnings, the run's duration and host, and SHA-256
                             digests of the inputs (CSR arrays, v0) and of the stored state

The GPU parity tests compare the library's result with these states element by element; they
recompute the input digests first, so a change of the generators cannot go unnoticed.  Nothing
here calls the HIP library: the expected values come from the oracle alone.
"""

import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def input_digest(H, v0: np.ndarray) -> str:
    """SHA-256 over the CSR arrays and the initial vector, in a fixed byte order."""
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(H.row_ptr, dtype="<i4"), np.ascontiguousarray(H.col, dtype="<i4"),
              np.ascontiguousarray(H.val, dtype="<c16"), np.ascontiguousarray(v0, dtype="<c16")):
        h.update(a.tobytes())
    return h.hexdigest()


def state_paths(name: str):
    return (os.path.join(HERE, f"oracle_state_{name}.npy"), os.path.join(HERE, f"oracle_state_{name}.json"))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make(name: str) -> dict:
    wl = workloads.workload(name)
    digest = input_digest(wl.H, wl.v0)
    t0 = time.time()

    def progress(steps, t_now, bound):
        print(f"  {name}: restart {steps}, t = {t_now:.6g} / {wl.t:g}, bound {bound:.3e}, "
              f"{time.time() - t0:.0f} s", flush=True)

    res = oracle.evolve(wl.H, wl.v0, wl.t, wl.tol, wl.m, on_step=progress)
    seconds = time.time() - t0
    v = np.ascontiguousarray(res.v, dtype="<c16")
    npy, meta_path = state_paths(name)
    np.save(npy, v)
    spec = workloads.WORKLOADS[name]
    meta = {
        "workload": name, "kind": spec["kind"], "size": spec["size"], "seed": spec["seed"],
        "dim": int(v.shape[0]), "nnz": int(wl.H.nnz), "t": wl.t, "tol": wl.tol, "m": wl.m,
        "steps": res.steps, "matvecs": res.matvecs, "err_bound": res.err_bound,
        "num_err_estimate": res.num_err_estimate, "warnings": res.warnings,
        "breakdown_dim": res.breakdown_dim, "t_reached": res.t_reached,
        "oracle_seconds": seconds, "host_cpu": cpu_model(), "host_threads": os.cpu_count(),
        "input_sha256": digest, "state_sha256": hashlib.sha256(v.tobytes()).hexdigest(),
        "taus": [s.tau for s in res.trace],
    }
    with open(meta_path, "w") as f:
        json.dump(meta, f, indent=1)
    print(f"{name}: {res.steps} restarts, bound {res.err_bound:.3e}, {seconds:.0f} s -> {npy}", flush=True)
    return meta


if __name__ == "__main__":
    names = sys.argv[1:] or ["xxz_L20"]
    for n in names:
        make(n)
