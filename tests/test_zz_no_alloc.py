"""te_evolve_noalloc (the evolution whose workspace is the library's static scratch array) against
te_evolve on the same handles and kernel shapes: bitwise equal states and equal result records,
on two calls in a row with the second one smaller, plus the host-side capacity check."""

import numpy as np
import pytest

import workloads
from gpu_util import announce, hamiltonian, lib, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

SHAPE = (1, 8, 4, 2, 0)  # lanes per row, nonzeros per lane, rows per thread, update rows, split


def _pair(L, seed, t, tol, m, shape=SHAPE, three_term=False):
    import torch
    te = lib()
    H, v0 = workloads.xxz_chain(L, seed=seed)
    opts = te.te_default_options(flags=te.TE_OPT_LANCZOS3 if three_term else 0)
    with hamiltonian(H) as h:
        te.te_set_tuning(h, *shape)
        x = to_dev(v0)
        announce(f"noalloc L={L} seed={seed} t={t} tol={tol} m={m} shape={shape} three_term={three_term}")
        ref, r_ref = te.te_evolve(h, x, t, tol, m, options=opts)
        out = torch.full_like(x, complex(float("nan"), float("nan")))
        got, r_got = te.te_evolve_noalloc(h, x, t, tol, m, out, options=opts)
        torch.cuda.synchronize()
    return to_host(ref), r_ref, to_host(got), r_got, v0


def _same(r1, r2):
    return ((r1.steps, r1.matvecs, r1.breakdown_dim, r1.warnings, r1.err_bound, r1.num_err_estimate, r1.t_reached)
            == (r2.steps, r2.matvecs, r2.breakdown_dim, r2.warnings, r2.err_bound, r2.num_err_estimate, r2.t_reached))


def test_noalloc_matches_te_evolve_twice_second_smaller():
    torch_dev()
    # first call: L = 16 (65,536 rows, 43 MB of basis at m = 40, most of the scratch array)
    ref, rr, got, rg, _ = _pair(16, 11, 10.0, 1e-8, 40)
    assert np.array_equal(ref, got)
    assert _same(rr, rg) and rg.steps > 1
    # second call, smaller: L = 10, another m; the array still holds the first call's basis
    ref, rr, got, rg, v0 = _pair(10, 12, 5.0, 1e-8, 30)
    assert np.array_equal(ref, got)
    assert _same(rr, rg) and rg.t_reached == 5.0
    assert abs(np.linalg.norm(got) - np.linalg.norm(v0)) <= rg.err_bound + 1e-12


def test_noalloc_other_shapes_and_three_term():
    torch_dev()
    for shape, tt in [((4, 4, 2, 1, 1), False), ((8, 2, 1, 2, 0), False), (SHAPE, True)]:
        ref, rr, got, rg, _ = _pair(12, 13, 10.0, 1e-8, 40, shape=shape, three_term=tt)
        assert np.array_equal(ref, got), shape
        assert _same(rr, rg)


def test_noalloc_capacity_and_arguments():
    import torch
    te = lib()
    torch_dev()
    H, v0 = workloads.xxz_chain(17, seed=14)  # 131,072 rows x 41 columns: 86 MB > 64 MiB
    with hamiltonian(H) as h:
        assert te.te_workspace_bytes(h, 40) + 256 > te.TE_NOALLOC_SCRATCH_BYTES
        te.te_set_tuning(h, *SHAPE)
        x = to_dev(v0)
        out = torch.empty_like(x)
        with pytest.raises(te.TEError) as e:
            te.te_evolve_noalloc(h, x, 1.0, 1e-8, 40, out)
        assert e.value.status == te.TE_ERR_CAPACITY
        with pytest.raises(te.TEError) as e:
            te.te_evolve_noalloc(h, x, 1.0, 1e-8, 40, out, options=te.te_default_options(flags=te.TE_OPT_PROFILE))
        assert e.value.status == te.TE_ERR_INVALID_ARG
        # a smaller m fits: 131,072 rows x 25 columns
        assert te.te_workspace_bytes(h, 24) + 256 <= te.TE_NOALLOC_SCRATCH_BYTES
        got, r = te.te_evolve_noalloc(h, x, 0.5, 1e-8, 24, out)
        ref, rr = te.te_evolve(h, x, 0.5, 1e-8, 24)
        assert np.array_equal(to_host(got), to_host(ref))
        assert _same(r, rr)
