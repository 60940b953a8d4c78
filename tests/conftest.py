import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The dense and sector references (eigh on a few hundred rows) run 50 times slower when a BLAS
# pool has more threads than free cores; four are enough for the test sizes.  NumPy and SciPy
# each load their own OpenBLAS: the variable covers both if set before they load, the limit
# below those already loaded.
_BLAS_THREADS = str(min(4, os.cpu_count() or 1))
os.environ.setdefault("OPENBLAS_NUM_THREADS", _BLAS_THREADS)
try:
    import numpy  # noqa: F401
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=int(os.environ["OPENBLAS_NUM_THREADS"]), user_api="blas")
except ImportError:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test (still part of the default CPU suite)")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible GPU; on a CPU-only host they are skipped, never silently
    # rerouted.  On a GPU host a missing library makes them fail (see tests/gpu_util.py).
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible on this host")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
