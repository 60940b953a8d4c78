"""MI355X-native restarted Krylov evolution exp(-iHt) v with a rigorous a-posteriori bound.

The computation lives in libtimeevolve.so (HIP for gfx950, C ABI in include/te.h); this
package only builds it (`build`), loads it (`te`, on first use: importing the package does
not touch the library, so it can be rebuilt in place) and offers convenience wrappers.
Using any of the names below without a built library raises ImportError.
"""

import importlib

_TE_NAMES = ("Hamiltonian", "TEError", "te_arnoldi", "te_default_options", "te_error_integral", "te_evolve",
             "te_hamiltonian_create", "te_last_profile", "te_autotune", "te_get_tuning", "te_set_tuning", "te_spmv", "te_step_search", "te_tridiag_eig",
             "te_workspace_bytes", "te_job_footprint", "te_evolve_sampled", "Engine", "te_batch_run", "te_engine_default_config",
             "te_hamiltonian_create_memory_burden", "te_memory_burden_defaults", "te_hamiltonian_copy_csr",
             "te_hamiltonian_create_bose_chain", "te_hamiltonian_pack")


def __getattr__(name):
    if name == "te":
        return importlib.import_module(".te", __name__)
    if name in _TE_NAMES:
        return getattr(importlib.import_module(".te", __name__), name)
    raise AttributeError(name)


def hamiltonian_from_csr(csr, check_hermitian=False, stream=None):
    """te_hamiltonian_create from any object with row_ptr / col / val host arrays."""
    te = importlib.import_module(".te", __name__)
    return te.te_hamiltonian_create(csr.row_ptr, csr.col, csr.val, check_hermitian=check_hermitian, stream=stream)


__all__ = list(_TE_NAMES) + ["te", "hamiltonian_from_csr"]
