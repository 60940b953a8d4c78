"""Helpers for the GPU tests: device tensors and a loud failure when the HIP library is missing."""

import numpy as np


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def lib():
    # raises ImportError (test failure) when libtimeevolve.so was not built: no fallback
    from paper_2205_15346_amd import te
    return te


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(torch_dev())


def to_host(t):
    return t.detach().cpu().numpy()


def hamiltonian(csr, check_hermitian=False):
    return lib().te_hamiltonian_create(csr.row_ptr, csr.col, csr.val, check_hermitian=check_hermitian)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
