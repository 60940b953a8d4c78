"""Named workloads: the single-solve configurations and the batch / serving draws.

single solves (Hamiltonian, v0, t, tol, m):
  xxz_L12   XXZ ring L=12 (d=4,096, nnz=28,672), seed 1, t=10,  tol=1e-8,  m=40
  xxz_L20   XXZ ring L=20 (d=1,048,576, nnz=11,534,336), seed 2, t=100, tol=1e-8, m=40
  bose_K12  Bose chain K=N=12 (d=1,352,078), seed 3, t=50, tol=1e-10, m=60
  paper_d1565904  the paper's performance example (Sec. "Analysis of Performance"): eq.
            fullHamiltonianSimple with K=K'=10, N_m=5, N_0=N_c=100 (d=1,565,904, 122,109,504
            stored entries), v0 of eq. initialStateSimple (no random draw: seed unused), t=10,
            err_max=1e-7, m=40
batch  (batch_jobs): 256 XXZ instances; master default_rng(4) draws per instance i, in
  this order, L=integers(10,19), n_v0=integers(1,9), t=uniform(1,100),
  tol=choice([1e-6,1e-8,1e-10]); the instance's H and its v0s come from seed 1000+i; m=40.
serving (serving_requests): master default_rng(5) draws per request r, in this order,
  gap=exponential(1/qps), kind=integers(0,2) (0: XXZ, 1: Bose),
  size=integers(14,23) for XXZ or integers(10,13) for Bose (N=K), t=uniform(1,100),
  tol=choice([1e-6,1e-10]); m=40.  The Hamiltonian of a (kind, size) pair is built once
  from seed 100000+size and shared by the requests that name it; request r draws its
  own v0 from seed 200000+r.
"""

from dataclasses import dataclass

import numpy as np

from .bosonic import bosonic_chain
from .csr import random_state
from .memory_burden import memory_burden_model
from .xxz import xxz_chain


@dataclass
class Workload:
    name: str
    H: object
    v0: np.ndarray
    t: float
    tol: float
    m: int


WORKLOADS = {
    "xxz_L12": dict(kind="xxz", size=12, seed=1, t=10.0, tol=1e-8, m=40),
    "xxz_L20": dict(kind="xxz", size=20, seed=2, t=100.0, tol=1e-8, m=40),
    "bose_K12": dict(kind="bose", size=12, seed=3, t=50.0, tol=1e-10, m=60),
    "paper_d1565904": dict(kind="memory_burden", size=10, seed=0, t=10.0, tol=1e-7, m=40),
}

# the paper's example: K = K' = size, N_m = size / 2, N_0 = N_c = 100
PAPER_MODEL_PARAMS = dict(K=10, Kp=10, Nm=5, N0=100, Nc=100.0)


def build_hamiltonian(kind: str, size: int, seed: int, with_v0: bool = True):
    if kind == "xxz":
        return xxz_chain(size, seed, with_v0=with_v0)
    if kind == "bose":
        return bosonic_chain(size, size, seed, with_v0=with_v0)
    if kind == "memory_burden":
        params = dict(PAPER_MODEL_PARAMS, K=size, Kp=size, Nm=size // 2)
        H, v0, _ = memory_burden_model(**params)
        return H, (v0 if with_v0 else None)
    raise ValueError(kind)


def workload(name: str) -> Workload:
    spec = WORKLOADS[name]
    H, v0 = build_hamiltonian(spec["kind"], spec["size"], spec["seed"])
    return Workload(name, H, v0, spec["t"], spec["tol"], spec["m"])


@dataclass
class BatchJob:
    index: int
    L: int
    n_v0: int
    t: float
    tol: float
    m: int = 40

    def build(self):
        """(H, [v0 ...]) for this instance, from seed 1000 + index."""
        H, vs = xxz_chain(self.L, 1000 + self.index, n_v0=self.n_v0)
        if self.n_v0 == 1:
            vs = [vs]
        return H, vs


def batch_jobs(n_instances: int = 256, seed: int = 4):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n_instances):
        L = int(rng.integers(10, 19))
        n_v0 = int(rng.integers(1, 9))
        t = float(rng.uniform(1.0, 100.0))
        tol = float(rng.choice([1e-6, 1e-8, 1e-10]))
        jobs.append(BatchJob(i, L, n_v0, t, tol))
    return jobs


@dataclass
class Request:
    index: int
    arrival: float
    kind: str
    size: int
    t: float
    tol: float
    m: int = 40

    def hamiltonian_key(self):
        return (self.kind, self.size)

    def v0(self, dim: int) -> np.ndarray:
        return random_state(np.random.default_rng(200000 + self.index), dim)


def serving_requests(n: int, qps: float, seed: int = 5, xxz_sizes=(14, 23), bose_sizes=(10, 13)):
    rng = np.random.default_rng(seed)
    now = 0.0
    out = []
    for r in range(n):
        now += float(rng.exponential(1.0 / qps))
        kind = "xxz" if int(rng.integers(0, 2)) == 0 else "bose"
        lo, hi = xxz_sizes if kind == "xxz" else bose_sizes
        size = int(rng.integers(lo, hi))
        t = float(rng.uniform(1.0, 100.0))
        tol = float(rng.choice([1e-6, 1e-10]))
        out.append(Request(r, now, kind, size, t, tol))
    return out


def serving_hamiltonian(kind: str, size: int):
    H, _ = build_hamiltonian(kind, size, 100000 + size, with_v0=False)
    return H
