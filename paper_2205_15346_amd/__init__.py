"""MI355X-native restarted Krylov evolution exp(-iHt) v with a rigorous a-posteriori bound.

The computation lives in libtimeevolve.so (HIP for gfx950, C ABI in include/te.h); this
package only loads it (`te`), builds it (`build`) and offers convenience wrappers.
"""

from . import te
from .te import (Hamiltonian, TEError, te_arnoldi, te_default_options, te_error_integral, te_evolve,
                 te_hamiltonian_create, te_spmv, te_step_search, te_tridiag_eig, te_workspace_bytes)


def hamiltonian_from_csr(csr, check_hermitian=False, stream=None) -> Hamiltonian:
    """te_hamiltonian_create from any object with row_ptr / col / val host arrays."""
    return te_hamiltonian_create(csr.row_ptr, csr.col, csr.val, check_hermitian=check_hermitian, stream=stream)


__all__ = [
    "te", "Hamiltonian", "TEError", "te_arnoldi", "te_default_options", "te_error_integral", "te_evolve",
    "te_hamiltonian_create", "te_spmv", "te_step_search", "te_tridiag_eig", "te_workspace_bytes",
    "hamiltonian_from_csr",
]
