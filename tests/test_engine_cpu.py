"""Host-side checks of the batched / served engine (no device needed): the pool allocator
(compiled from the engine's own header with g++ and exercised against a bitmap model), the
job footprint used for admission, the default configuration and argument validation."""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_15346_amd", "csrc")


def test_pool_allocator_against_model(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "pool_test")
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "pool_test.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "pool ok" in out.stdout


def _units(n):
    return (n + 255) // 256 * 256


@pytest.mark.parametrize("dim,m", [(1, 40), (100, 40), (1024, 40), (262144, 40), (4194304, 40), (1352078, 60)])
def test_job_footprint(dim, m):
    from paper_2205_15346_amd import te
    mm = min(m, dim)
    ld = (dim + 63) // 64 * 64
    tiles = (dim + 255) // 256
    expect = (_units(mm * ld * 16) + _units(ld * 16) + _units(130 * tiles * 16) + _units(tiles * 8)
              + _units(130 * 16))
    assert te.te_job_footprint(dim, m) == expect
    # basis and product vector dominate; partials add 130 * 16 / 256 bytes per row
    assert expect <= (mm + 1) * 16 * ld + 8.2 * ld + (64 << 10)


def test_footprint_invalid_and_monotone():
    from paper_2205_15346_amd import te
    assert te.te_job_footprint(0, 40) == 0
    assert te.te_job_footprint(100, 0) == 0
    assert te.te_job_footprint(100, 65) == 0
    assert te.te_job_footprint(1 << 31, 40) == 0
    sizes = [te.te_job_footprint(1 << L, 40) for L in range(10, 23)]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    # an XXZ L=22 job: 40 basis columns + product vector of 4,194,304 complex numbers
    assert 2.7e9 < te.te_job_footprint(1 << 22, 40) < 2.9e9


def test_default_config():
    from paper_2205_15346_amd import te
    c = te.te_engine_default_config()
    assert (c.m, c.max_jobs, c.hbm_budget, c.lanes_per_row, c.nnz_per_lane, c.rows_per_thread,
            c.update_rows_per_thread, c.flags) == (40, 1024, 0, 0, 0, 0, 0, te.TE_ENGINE_THREADED)
    assert c.opt.n_substeps == 10 and c.opt.shrink == 0.97
    assert (c.lane_rows, c.lane_jobs) == (0, 0)  # one lane unless asked


@pytest.mark.parametrize("field,value,status", [
    ("m", 1, "TE_ERR_INVALID_ARG"), ("m", 65, "TE_ERR_UNSUPPORTED"), ("max_jobs", 0, "TE_ERR_INVALID_ARG"),
    ("max_jobs", 16385, "TE_ERR_INVALID_ARG"), ("lanes_per_row", 3, "TE_ERR_INVALID_ARG"),
    ("update_rows_per_thread", 3, "TE_ERR_INVALID_ARG"), ("rows_per_thread", 3, "TE_ERR_INVALID_ARG"),
    ("flags", 8, "TE_ERR_INVALID_ARG"),
    ("hbm_budget", 0, "TE_ERR_INVALID_ARG"), ("lane_rows", -1, "TE_ERR_INVALID_ARG"),
    ("lane_jobs", -1, "TE_ERR_INVALID_ARG"), ("lane_jobs", 1025, "TE_ERR_INVALID_ARG")])
def test_engine_create_validates_before_touching_the_device(field, value, status):
    from paper_2205_15346_amd import te
    c = te.te_engine_default_config(hbm_budget=1 << 30)
    setattr(c, field, value)
    e = ctypes.c_void_p()
    assert te._lib.te_engine_create(ctypes.byref(e), ctypes.byref(c), None) == getattr(te, status)
    assert e.value is None
    assert te._lib.te_last_error()


def test_engine_calls_reject_null_handles():
    from paper_2205_15346_amd import te
    lib = te._lib
    jid = ctypes.c_int64()
    assert lib.te_engine_submit(None, None, None, None, 1.0, 1e-8, ctypes.byref(jid)) == te.TE_ERR_INVALID_ARG
    assert lib.te_engine_poll(None, 0, None, None) == te.TE_ERR_INVALID_ARG
    assert lib.te_engine_wait(None, -1, 0.0) == te.TE_ERR_INVALID_ARG
    assert lib.te_engine_get_stats(None, None) == te.TE_ERR_INVALID_ARG
    assert lib.te_engine_destroy(None) == te.TE_ERR_INVALID_ARG


def test_batch_host_calls():
    from paper_2205_15346_amd import te
    lib = te._lib
    c = te.te_engine_default_config()
    b = ctypes.c_void_p()
    assert lib.te_batch_create(ctypes.byref(b), ctypes.byref(c), None) == te.TE_OK
    try:
        first = ctypes.c_int32()
        ptrs = (ctypes.c_void_p * 1)(None)
        assert lib.te_batch_add(b, None, 1, ptrs, ptrs, 1.0, 1e-8, ctypes.byref(first)) == te.TE_ERR_INVALID_ARG
        r = te.te_result()
        s = ctypes.c_int32()
        assert lib.te_batch_result(b, 0, ctypes.byref(r), ctypes.byref(s)) == te.TE_ERR_INVALID_ARG
    finally:
        assert lib.te_batch_destroy(b) == te.TE_OK
    c.m = 1
    assert lib.te_batch_create(ctypes.byref(b), ctypes.byref(c), None) == te.TE_ERR_INVALID_ARG
