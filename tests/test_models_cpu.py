"""Host side of the device-built exemplary Hamiltonian: the C defaults are the paper's Fig. 1
system (the same parameters the host workload builder uses), and out-of-range parameters are
rejected before any device work (these run without a GPU)."""

import ctypes

import numpy as np
import pytest

from workloads import memory_burden as MB


def test_defaults_are_the_papers_system():
    from paper_2205_15346_amd import te
    p = te.te_memory_burden_defaults()
    D = MB.DEFAULTS
    assert (p.K, p.Kp, p.N0, p.Nm) == (D["K"], D["Kp"], D["N0"], D["Nm"])
    assert (p.eps_m, p.Nc, p.dNc, p.C0, p.Cm) == (D["eps_m"], D["Nc"], D["dNc"], D["C0"], D["Cm"])
    assert MB.memory_burden_dim(p.N0, p.K, p.Kp, p.Nm) == 588


@pytest.mark.parametrize("field,value,status", [
    ("K", 0, "TE_ERR_INVALID_ARG"), ("Kp", -1, "TE_ERR_INVALID_ARG"), ("Nm", 5, "TE_ERR_INVALID_ARG"),
    ("N0", -1, "TE_ERR_INVALID_ARG"), ("dNc", 0.0, "TE_ERR_INVALID_ARG"), ("dNc", 20.0, "TE_ERR_INVALID_ARG"),
    ("eps_m", float("nan"), "TE_ERR_INVALID_ARG"), ("Kp", 60, "TE_ERR_INVALID_ARG")])
def test_out_of_range_parameters_are_rejected(field, value, status):
    from paper_2205_15346_amd import te
    p = te.te_memory_burden_defaults()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    assert te._lib.te_hamiltonian_create_memory_burden(ctypes.byref(h), ctypes.byref(p), None, None) == \
        getattr(te, status)
    assert h.value is None and te._lib.te_last_error()


@pytest.mark.parametrize("params", [dict(K=16, Kp=16, Nm=16, N0=0), dict(K=20, Kp=20, Nm=10, N0=2000)])
def test_sizes_beyond_int32_or_row_slots_are_unsupported(params):
    from paper_2205_15346_amd import te
    p = te.te_memory_burden_defaults(**params)
    h = ctypes.c_void_p()
    assert te._lib.te_hamiltonian_create_memory_burden(ctypes.byref(h), ctypes.byref(p), None, None) == \
        te.TE_ERR_UNSUPPORTED
