"""CPU checks of the C ABI: the library loads, exports every function include/te.h declares,
and the host-only calls (defaults, status strings, sizes, argument validation) behave."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "te.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:te_status|void|size_t|uint64_t|const char\*)\s+(te_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ["te_hamiltonian_create", "te_hamiltonian_destroy", "te_hamiltonian_info", "te_evolve",
                     "te_workspace_bytes", "te_spmv", "te_arnoldi", "te_tridiag_eig", "te_error_integral",
                     "te_step_search", "te_status_string", "te_last_error", "te_default_options",
                     "te_set_allocator"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2205_15346_amd import te
    lib = ctypes.CDLL(te.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    assert sorted(te.exported_symbols()) == header_functions()


def test_host_only_calls():
    from paper_2205_15346_amd import te
    o = te.te_default_options()
    assert (o.n_substeps, o.t_init, o.shrink, o.quad_rel_tol, o.quad_max_level, o.quad_min_level,
            o.max_halvings, o.flags, o.quad_gauss_points) == (10, 0.1, 0.97, 1e-3, 15, 3, 64, 0, 0)
    assert te.te_status_string(te.TE_OK) == "ok"
    assert "step" in te.te_status_string(te.TE_ERR_STEP_UNDERFLOW)
    # the workspace size needs a handle (sizes with one are checked by the GPU tests)
    assert te.te_workspace_bytes(None, 40) == 0


def test_argument_validation_without_device():
    from paper_2205_15346_amd import te
    lib = te._lib
    assert lib.te_evolve(None, None, None, 1.0, 1e-8, 10, None, None, None) == te.TE_ERR_INVALID_ARG
    assert b"null" in lib.te_last_error()
    a = (ctypes.c_double * 2)()
    assert lib.te_tridiag_eig(0, a, a, a, a, None) == te.TE_ERR_INVALID_ARG
    assert lib.te_tridiag_eig(65, a, a, a, a, None) == te.TE_ERR_INVALID_ARG
    nan = (ctypes.c_double * 2)(float("nan"), 0.0)
    assert lib.te_tridiag_eig(2, nan, a, a, a, None) == te.TE_ERR_NONFINITE
    assert lib.te_hamiltonian_create(None, 10, 10, None, None, None, 0, None) == te.TE_ERR_INVALID_ARG
    assert lib.te_set_allocator(ctypes.c_void_p(1), None, None) == te.TE_ERR_INVALID_ARG
    assert lib.te_set_allocator(None, None, None) == te.TE_OK


def test_product_path_has_no_oracle_dependency():
    # the package must not import, load or run anything from oracle/
    pkg = os.path.join(ROOT, "paper_2205_15346_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
