"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This package only *constructs inputs* (Hamiltonian matrices in CSR form and
initial vectors).  It contains none of the time-evolution arithmetic, so both
the oracle and the HIP path may import it without sharing any of the method.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed, documented order, so a (model, size, seed) triple names one input.
"""

from .csr import CSR, random_state
from .xxz import xxz_chain, xxz_nnz
from .bosonic import bose_chain_params, bosonic_chain, fock_basis, fock_dim, capped_fock_basis
from .memory_burden import memory_burden_model, memory_burden_dim
from .configs import PAPER_MODEL_PARAMS, workload, WORKLOADS, batch_jobs, serving_requests

__all__ = [
    "CSR", "random_state", "xxz_chain", "xxz_nnz", "bosonic_chain", "bose_chain_params", "fock_basis",
    "fock_dim", "capped_fock_basis", "memory_burden_model", "memory_burden_dim",
    "PAPER_MODEL_PARAMS", "workload", "WORKLOADS", "batch_jobs", "serving_requests",
]
