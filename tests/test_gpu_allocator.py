"""te_set_allocator with PyTorch's caching allocator as the library's device allocator: the
evolution and the engine give bitwise the results they give on hipMalloc memory, every block
the library takes goes back, and te_evolve_noalloc takes none."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import announce, hamiltonian, lib, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu
SHAPE = (1, 8, 4, 2, 0)


class Counting:
    """PyTorch's caching allocator behind counters of the library's calls."""

    def __init__(self):
        te = lib()
        self.alloc_fn, self.free_fn = te.torch_caching_allocator()
        self.live = {}
        self.allocs = 0
        self.frees = 0
        self.streams = set()

    def alloc(self, nbytes, stream):
        p = self.alloc_fn(nbytes, stream)
        self.allocs += 1
        self.live[p] = nbytes
        self.streams.add(stream)
        return p

    def free(self, ptr, stream):
        assert ptr in self.live, "freed a block this allocator did not supply"
        del self.live[ptr]
        self.frees += 1
        self.free_fn(ptr, stream)


def run_evolve(H, v0, t, tol, m):
    te = lib()
    with hamiltonian(H) as h:
        te.te_set_tuning(h, *SHAPE)
        out, res = te.te_evolve(h, to_dev(v0), t, tol, m)
        return to_host(out), res


def run_engine(jobs):
    te = lib()
    hs = [hamiltonian(H) for H, _, _, _ in jobs]
    budget = 4 * max(te.te_job_footprint(H.dim, 40) for H, _, _, _ in jobs)
    outs = []
    with te.Engine(budget, m=40, shape=(1, 8), rows_per_thread=4, update_rows_per_thread=2) as eng:
        ids = [eng.submit(h, to_dev(v0), t, tol) for h, (_, v0, t, tol) in zip(hs, jobs)]
        eng.wait()
        for j in ids:
            info, res = eng.poll(j)
            outs.append((to_host(eng.output(j)), res.err_bound, res.steps))
    for h in hs:
        h.destroy()
    return outs


def test_torch_caching_allocator_bitwise():
    import torch
    te = lib()
    torch_dev()
    H, v0 = W.xxz_chain(14, seed=31)
    Hb, vb = W.bosonic_chain(6, 6, seed=32)
    jobs = [(H, v0, 3.0, 1e-8), (Hb, vb, 2.0, 1e-10), (H, W.random_state(np.random.default_rng(33), H.dim), 1.0, 1e-6)]
    announce("allocator: reference runs on hipMalloc")
    ref_v, ref_r = run_evolve(H, v0, 5.0, 1e-8, 40)
    ref_jobs = run_engine(jobs)
    cnt = Counting()
    te.te_set_allocator(cnt.alloc, cnt.free)
    try:
        announce("allocator: te_evolve and an engine on PyTorch's caching allocator")
        v, r = run_evolve(H, v0, 5.0, 1e-8, 40)
        got_jobs = run_engine(jobs)
        assert cnt.allocs > 0 and cnt.frees == cnt.allocs and not cnt.live
        # te_evolve_noalloc takes nothing from the allocator (the handle's own copy aside)
        with hamiltonian(H) as h:
            te.te_set_tuning(h, *SHAPE)
            x = to_dev(v0)
            out = torch.empty_like(x)
            a0 = cnt.allocs
            got, rn = te.te_evolve_noalloc(h, x, 5.0, 1e-8, 40, out)
            assert cnt.allocs == a0
            assert np.array_equal(to_host(got), ref_v)
    finally:
        te.te_set_allocator(None, None)
    assert np.array_equal(v, ref_v)
    assert (r.steps, r.err_bound) == (ref_r.steps, ref_r.err_bound)
    for (a, ea, sa), (b, eb, sb) in zip(got_jobs, ref_jobs):
        assert np.array_equal(a, b) and ea == eb and sa == sb


def test_blocks_return_to_their_allocator_after_a_switch():
    import torch
    te = lib()
    torch_dev()
    H, v0 = W.xxz_chain(10, seed=34)
    cnt = Counting()
    te.te_set_allocator(cnt.alloc, cnt.free)
    try:
        h = hamiltonian(H)  # matrix copies from the hook
    finally:
        te.te_set_allocator(None, None)
    held = dict(cnt.live)  # the matrix (creation's own scratch has gone back already)
    assert held and cnt.frees == cnt.allocs - len(held)
    # the workspace now comes from hipMalloc, the matrix still belongs to the hook
    out, res = te.te_evolve(h, to_dev(v0), 1.0, 1e-8, 20)
    assert res.t_reached == 1.0
    assert cnt.live == held
    h.destroy()
    assert cnt.frees == cnt.allocs and not cnt.live
    torch.cuda.synchronize()
