"""Thin Python binding of libtimeevolve (include/te.h): argument marshalling only.

Every function carries the C name and forwards to the HIP library; device buffers are
torch.complex128 / float64 tensors on the current HIP device, and the current torch stream is
passed as the hipStream_t.  There is no fallback: if the library is missing this module
raises at import time.
"""

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtimeevolve.so")

TE_OK = 0
TE_ERR_INVALID_ARG = 1
TE_ERR_INVALID_CSR = 2
TE_ERR_NOT_HERMITIAN = 3
TE_ERR_UNSUPPORTED = 4
TE_ERR_OUT_OF_MEMORY = 5
TE_ERR_DEVICE = 6
TE_ERR_STEP_UNDERFLOW = 7
TE_ERR_NONFINITE = 8
TE_ERR_CAPACITY = 9
TE_ERR_TIMEOUT = 10
TE_WARN_NUMERICAL = 1
TE_WARN_QUADRATURE = 2
TE_PTR_DEVICE = 1
TE_CHECK_HERMITIAN = 2
TE_STORE_COMPLEX = 4
TE_STORE_CSR = 8
TE_STORAGE_COMPLEX, TE_STORAGE_REAL, TE_STORAGE_PACKED8, TE_STORAGE_PACKED16 = 0, 1, 2, 3
TE_STORAGE_CODED8, TE_STORAGE_CODED16 = 4, 5
STORAGE_NAMES = {0: "complex", 1: "real", 2: "packed8", 3: "packed16", 4: "coded8", 5: "coded16"}
TE_MAX_KRYLOV = 64
TE_NOALLOC_SCRATCH_BYTES = 64 << 20


class te_c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class te_options(ctypes.Structure):
    _fields_ = [("n_substeps", ctypes.c_int32), ("t_init", ctypes.c_double), ("shrink", ctypes.c_double),
                ("quad_rel_tol", ctypes.c_double), ("quad_max_level", ctypes.c_int32),
                ("quad_min_level", ctypes.c_int32), ("max_halvings", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("quad_gauss_points", ctypes.c_int32)]


class te_result(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("breakdown_dim", ctypes.c_int32),
                ("warnings", ctypes.c_uint32), ("err_bound", ctypes.c_double),
                ("num_err_estimate", ctypes.c_double), ("t_reached", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


TE_OPT_PROFILE = 1
TE_OPT_LANCZOS3 = 2
KERNEL_CLASSES = ("project", "update", "step", "combine", "fold")


class te_memory_burden(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Kp", ctypes.c_int32), ("N0", ctypes.c_int32), ("Nm", ctypes.c_int32),
                ("eps_m", ctypes.c_double), ("Nc", ctypes.c_double), ("dNc", ctypes.c_double),
                ("C0", ctypes.c_double), ("Cm", ctypes.c_double)]


class te_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 5), ("seconds", ctypes.c_double * 5), ("bytes", ctypes.c_double * 5)]

    def as_dict(self):
        return {name: {"launches": int(self.launches[i]), "seconds": float(self.seconds[i]),
                       "bytes": float(self.bytes[i])} for i, name in enumerate(KERNEL_CLASSES)}


class te_tuning(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_int32), ("nnz_per_lane", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32), ("update_rows_per_thread", ctypes.c_int32),
                ("split_projection", ctypes.c_int32), ("project_us", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


TE_ENGINE_THREADED = 1
TE_ENGINE_PROFILE = 2
TE_JOB_QUEUED, TE_JOB_RUNNING, TE_JOB_DONE, TE_JOB_FAILED = 0, 1, 2, 3
JOB_STATES = ("queued", "running", "done", "failed")


class te_engine_config(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("max_jobs", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("lanes_per_row", ctypes.c_int32), ("nnz_per_lane", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32), ("update_rows_per_thread", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("opt", te_options), ("lane_rows", ctypes.c_int64),
                ("lane_jobs", ctypes.c_int32)]


class te_job_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("t_now", ctypes.c_double), ("submitted", ctypes.c_double),
                ("admitted", ctypes.c_double), ("finished", ctypes.c_double)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["state"] = JOB_STATES[self.state]
        return d


class te_engine_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("plans", ctypes.c_int64), ("jobs_submitted", ctypes.c_int64),
                ("jobs_done", ctypes.c_int64), ("jobs_failed", ctypes.c_int64), ("jobs_queued", ctypes.c_int64),
                ("jobs_running", ctypes.c_int64), ("pool_bytes", ctypes.c_uint64), ("pool_used", ctypes.c_uint64),
                ("pool_peak", ctypes.c_uint64), ("busy_seconds", ctypes.c_double), ("tuning", te_tuning),
                ("prof", te_profile)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in ("tuning", "prof")}
        d["tuning"] = self.tuning.as_dict()
        d["prof"] = self.prof.as_dict()
        return d


class te_samples(ctypes.Structure):
    _fields_ = [("n_times", ctypes.c_int32), ("times", ctypes.c_void_p), ("states", ctypes.c_void_p),
                ("n_obs", ctypes.c_int32), ("obs", ctypes.c_void_p), ("obs_out", ctypes.c_void_p),
                ("bound_out", ctypes.c_void_p)]


class TEError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libtimeevolve.so is not built ({LIB_PATH}); run `python -m paper_2205_15346_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32
_I64 = ctypes.c_int64
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int32)
_PU = ctypes.POINTER(ctypes.c_uint32)

_SIGS = {
    "te_default_options": (None, [ctypes.POINTER(te_options)]),
    "te_status_string": (ctypes.c_char_p, [_I]),
    "te_last_error": (ctypes.c_char_p, []),
    "te_hamiltonian_create": (_I, [ctypes.POINTER(_P), _I64, _I64, _P, _P, _P, ctypes.c_uint32, _P]),
    "te_hamiltonian_destroy": (_I, [_P]),
    "te_hamiltonian_info": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _PD]),
    "te_hamiltonian_real_values": (_I, [_P, _PI]),
    "te_hamiltonian_storage": (_I, [_P, _PI]),
    "te_hamiltonian_pack": (_I, [_P, _PI, _P]),
    "te_hamiltonian_copy_csr": (_I, [_P, _P, _P, _P, ctypes.c_uint32, _P]),
    "te_memory_burden_defaults": (None, [ctypes.c_void_p]),
    "te_hamiltonian_create_memory_burden": (_I, [ctypes.POINTER(_P), ctypes.c_void_p, ctypes.POINTER(_I64), _P]),
    "te_hamiltonian_create_bose_chain": (_I, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, _P, _P,
                                              ctypes.c_uint32, _P]),
    "te_workspace_bytes": (ctypes.c_size_t, [_P, _I]),
    "te_set_allocator": (_I, [_P, _P, _P]),
    "te_evolve": (_I, [_P, _P, _P, _D, _D, _I, ctypes.POINTER(te_options), ctypes.POINTER(te_result), _P]),
    "te_evolve_noalloc": (_I, [_P, _P, _P, _D, _D, _I, ctypes.POINTER(te_options), ctypes.POINTER(te_result),
                               _P]),
    "te_last_profile": (_I, [_P, ctypes.POINTER(te_profile)]),
    "te_evolve_sampled": (_I, [_P, _P, _P, _D, _D, _I, ctypes.POINTER(te_options), ctypes.POINTER(te_samples),
                               ctypes.POINTER(te_result), _P]),
    "te_autotune": (_I, [_P, _I, ctypes.POINTER(te_tuning), _P]),
    "te_get_tuning": (_I, [_P, ctypes.POINTER(te_tuning)]),
    "te_set_tuning": (_I, [_P, ctypes.POINTER(te_tuning)]),
    "te_spmv": (_I, [_P, _P, _P, ctypes.POINTER(te_c128), _P]),
    "te_arnoldi": (_I, [_P, _P, _I, _D, _P, _PD, _PD, _PI, _P]),
    "te_tridiag_eig": (_I, [_I, _PD, _PD, _PD, _PD, _P]),
    "te_error_integral": (_I, [_I, _PD, _PD, _D, _D, _D, ctypes.POINTER(te_options), _PD, _PI, _PI, _P]),
    "te_step_search": (_I, [_I, _PD, _PD, _D, _D, _D, _I, _D, _I, ctypes.POINTER(te_options), _PD, _PD,
                            ctypes.POINTER(te_c128), _PU, _P]),
    "te_job_footprint": (ctypes.c_uint64, [_I64, _I]),
    "te_engine_default_config": (None, [ctypes.POINTER(te_engine_config)]),
    "te_engine_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(te_engine_config), _P]),
    "te_engine_submit": (_I, [_P, _P, _P, _P, _D, _D, ctypes.POINTER(_I64)]),
    "te_engine_poll": (_I, [_P, _I64, ctypes.POINTER(te_job_info), ctypes.POINTER(te_result)]),
    "te_engine_wait": (_I, [_P, _I64, _D]),
    "te_engine_get_stats": (_I, [_P, ctypes.POINTER(te_engine_stats)]),
    "te_engine_destroy": (_I, [_P]),
    "te_batch_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(te_engine_config), _P]),
    "te_batch_add": (_I, [_P, _P, _I, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _D, _PI]),
    "te_batch_launch": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(te_engine_stats)]),
    "te_batch_result": (_I, [_P, _I, ctypes.POINTER(te_result), _PI]),
    "te_batch_info": (_I, [_P, _I, ctypes.POINTER(te_job_info)]),
    "te_batch_destroy": (_I, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(status):
    if status != TE_OK:
        raise TEError(status, _lib.te_last_error().decode() or _lib.te_status_string(status).decode())


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_c128(t, name, dim=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous complex128 CUDA tensor")
    if dim is not None and t.numel() != dim:
        raise ValueError(f"{name} must have {dim} elements")
    return ctypes.c_void_p(t.data_ptr())


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_PD)


def te_default_options(**overrides) -> te_options:
    o = te_options()
    _lib.te_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def te_status_string(status: int) -> str:
    return _lib.te_status_string(status).decode()


def te_workspace_bytes(H, m: int) -> int:
    """Device bytes te_evolve keeps in handle H for Krylov dimension m (0 for H = None)."""
    return int(_lib.te_workspace_bytes(H.handle if H is not None else None, int(m)))


TE_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
TE_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator_callbacks = []  # installed callbacks stay alive: blocks they supplied may be freed later


def te_set_allocator(alloc=None, free=None):
    """Installs alloc(nbytes, stream) -> device address (int, 0 on failure) and
    free(address, stream) as the library's device allocator; both None restore hipMalloc/hipFree.
    ``stream`` is the raw hipStream_t value (0 = default stream)."""
    if alloc is None and free is None:
        _check(_lib.te_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("alloc and free must be given together")

    def _alloc(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:
            return None  # the library reports TE_ERR_OUT_OF_MEMORY

    def _free(ptr, stream, ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:
            pass

    ca, cf = TE_ALLOC_FN(_alloc), TE_FREE_FN(_free)
    _allocator_callbacks.append((ca, cf))
    _check(_lib.te_set_allocator(ctypes.cast(ca, ctypes.c_void_p), ctypes.cast(cf, ctypes.c_void_p), None))


def torch_caching_allocator(device=None):
    """(alloc, free) for te_set_allocator over PyTorch's caching allocator on one device."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, dev, stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


class Hamiltonian:
    """Owner of a te_hamiltonian handle (te_hamiltonian_create / te_hamiltonian_destroy)."""

    def __init__(self, handle):
        self._h = handle
        dim, nnz, n1 = _I64(), _I64(), _D()
        _check(_lib.te_hamiltonian_info(self._h, ctypes.byref(dim), ctypes.byref(nnz), ctypes.byref(n1)))
        self.dim, self.nnz, self.norm1 = dim.value, nnz.value, n1.value
        rv = _I()
        _check(_lib.te_hamiltonian_real_values(self._h, ctypes.byref(rv)))
        self.real_values = bool(rv.value)  # entries stored as real (8 B) rather than complex
        sk = ctypes.c_int32()
        _check(_lib.te_hamiltonian_storage(self._h, ctypes.byref(sk)))
        self.storage = STORAGE_NAMES[sk.value]  # "complex", "real", "packed8/16" or "coded8/16"

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("Hamiltonian already destroyed")
        return self._h

    def destroy(self):
        if self._h is not None:
            _check(_lib.te_hamiltonian_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def te_hamiltonian_create(row_ptr, col_idx, values, check_hermitian=False, stream=None,
                          store_complex=False, store_csr=False) -> Hamiltonian:
    """From host NumPy arrays (int32, int32, complex128) or CUDA tensors of the same dtypes.
    Entries are packed (codes into a table of (column offset, value) pairs) when few distinct
    pairs occur, unless store_csr is set; else a matrix whose imaginary parts are all zero is
    stored with real entries unless store_complex is set."""
    import torch
    flags = ((TE_CHECK_HERMITIAN if check_hermitian else 0) | (TE_STORE_COMPLEX if store_complex else 0)
             | (TE_STORE_CSR if store_csr else 0))
    keep = []
    if isinstance(values, torch.Tensor):
        flags |= TE_PTR_DEVICE
        rp, ci, va = row_ptr.contiguous(), col_idx.contiguous(), values.contiguous()
        if rp.dtype != torch.int32 or ci.dtype != torch.int32 or va.dtype != torch.complex128:
            raise TypeError("device CSR needs int32, int32, complex128 tensors")
        keep += [rp, ci, va]
        ptrs = [ctypes.c_void_p(x.data_ptr()) for x in (rp, ci, va)]
        dim, nnz = rp.numel() - 1, ci.numel()
    else:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.complex128)
        keep += [rp, ci, va]
        ptrs = [ctypes.c_void_p(x.ctypes.data) for x in (rp, ci, va)]
        dim, nnz = rp.size - 1, ci.size
    h = _P()
    _check(_lib.te_hamiltonian_create(ctypes.byref(h), dim, nnz, *ptrs, flags, _stream(stream)))
    return Hamiltonian(h)


def te_memory_burden_defaults(**overrides) -> te_memory_burden:
    p = te_memory_burden()
    _lib.te_memory_burden_defaults(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def te_hamiltonian_create_memory_burden(model=None, stream=None, **overrides):
    """The paper's exemplary Hamiltonian built on the device; returns (Hamiltonian, index of
    the initial state).  Parameters: a te_memory_burden, else the defaults with overrides."""
    p = model if model is not None else te_memory_burden_defaults(**overrides)
    h, idx = _P(), _I64()
    _check(_lib.te_hamiltonian_create_memory_burden(ctypes.byref(h), ctypes.byref(p), ctypes.byref(idx),
                                                    _stream(stream)))
    return Hamiltonian(h), idx.value


def te_hamiltonian_create_bose_chain(U, hop, N: int, store_complex=False, stream=None) -> Hamiltonian:
    """Open Bose chain of len(U) modes and N bosons built on the device: hop[k] couples modes k
    and k + 1 (len(hop) = len(U) - 1), U[k] n_k (n_k - 1) on site."""
    u = np.ascontiguousarray(U, dtype=np.float64)
    a = np.ascontiguousarray(hop, dtype=np.complex128)
    if u.ndim != 1 or a.shape != (max(u.size - 1, 0),):
        raise ValueError("need len(hop) == len(U) - 1")
    h = _P()
    flags = TE_STORE_COMPLEX if store_complex else 0
    _check(_lib.te_hamiltonian_create_bose_chain(ctypes.byref(h), int(u.size), int(N), ctypes.c_void_p(u.ctypes.data),
                                                 ctypes.c_void_p(a.ctypes.data) if a.size else None, flags,
                                                 _stream(stream)))
    return Hamiltonian(h)


def te_hamiltonian_pack(H: Hamiltonian, stream=None) -> str:
    """Packs a CSR handle's entries in place (as creation would); returns the storage name."""
    k = ctypes.c_int32()
    _check(_lib.te_hamiltonian_pack(H.handle, ctypes.byref(k), _stream(stream)))
    H.storage = STORAGE_NAMES[k.value]
    H.real_values = H.storage == "real"
    return H.storage


def te_hamiltonian_copy_csr(H: Hamiltonian, stream=None):
    """Host copies (row_ptr int32, col int32, values complex128) of the handle's matrix."""
    rp = np.empty(H.dim + 1, dtype=np.int32)
    ci = np.empty(H.nnz, dtype=np.int32)
    va = np.empty(H.nnz, dtype=np.complex128)
    _check(_lib.te_hamiltonian_copy_csr(H.handle, ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(ci.ctypes.data),
                                        ctypes.c_void_p(va.ctypes.data), 0, _stream(stream)))
    return rp, ci, va


def te_evolve(H: Hamiltonian, v0, t: float, tol: float, m: int, options=None, out=None, stream=None):
    """v(t) = exp(-iHt) v0; returns (v_out tensor, te_result)."""
    import torch
    p0 = _dev_c128(v0, "v0", H.dim)
    if out is None:
        out = torch.empty_like(v0)
    p1 = _dev_c128(out, "out", H.dim)
    res = te_result()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.te_evolve(H.handle, p0, p1, float(t), float(tol), int(m), opt, ctypes.byref(res), _stream(stream)))
    return out, res


def te_evolve_noalloc(H: Hamiltonian, v0, t: float, tol: float, m: int, out, options=None, stream=None):
    """te_evolve with the workspace in the library's static per-device scratch array (no device
    allocation by the library); ``out`` must be given.  Returns (out, te_result)."""
    p0 = _dev_c128(v0, "v0", H.dim)
    p1 = _dev_c128(out, "out", H.dim)
    res = te_result()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.te_evolve_noalloc(H.handle, p0, p1, float(t), float(tol), int(m), opt, ctypes.byref(res),
                                  _stream(stream)))
    return out, res


def te_evolve_sampled(H: Hamiltonian, v0, t: float, tol: float, m: int, times, states=True, obs=None,
                      options=None, out=None, stream=None):
    """v(t) plus the states and/or diagonal observables at the given times: returns
    (v_out tensor, te_result, states tensor [n, dim] or None, observables [n, n_obs] or None,
    bounds [n])."""
    import torch
    p0 = _dev_c128(v0, "v0", H.dim)
    if out is None:
        out = torch.empty_like(v0)
    p1 = _dev_c128(out, "out", H.dim)
    ts = np.ascontiguousarray(times, dtype=np.float64)
    n = ts.size
    st = torch.empty((n, H.dim), dtype=torch.complex128, device=v0.device) if states else None
    n_obs = 0
    obs_out = None
    if obs is not None:
        if not (isinstance(obs, torch.Tensor) and obs.is_cuda and obs.dtype == torch.float64 and obs.is_contiguous()
                and obs.dim() == 2 and obs.shape[1] == H.dim):
            raise TypeError("obs must be a contiguous float64 CUDA tensor [n_obs, dim]")
        n_obs = obs.shape[0]
        obs_out = np.zeros((n, n_obs))
    bounds = np.zeros(n)
    smp = te_samples(n, ts.ctypes.data, st.data_ptr() if st is not None else None, n_obs,
                     obs.data_ptr() if obs is not None else None,
                     obs_out.ctypes.data if obs_out is not None else None, bounds.ctypes.data)
    res = te_result()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.te_evolve_sampled(H.handle, p0, p1, float(t), float(tol), int(m), opt, ctypes.byref(smp),
                                  ctypes.byref(res), _stream(stream)))
    return out, res, st, obs_out, bounds


def te_autotune(H: Hamiltonian, m: int, stream=None) -> te_tuning:
    t = te_tuning()
    _check(_lib.te_autotune(H.handle, int(m), ctypes.byref(t), _stream(stream)))
    return t


def te_get_tuning(H: Hamiltonian) -> te_tuning:
    t = te_tuning()
    _check(_lib.te_get_tuning(H.handle, ctypes.byref(t)))
    return t


def te_set_tuning(H: Hamiltonian, lanes_per_row, nnz_per_lane, rows_per_thread, update_rows_per_thread,
                  split_projection=0):
    t = te_tuning(lanes_per_row, nnz_per_lane, rows_per_thread, update_rows_per_thread, split_projection, 0.0)
    _check(_lib.te_set_tuning(H.handle, ctypes.byref(t)))


def te_last_profile(H: Hamiltonian) -> te_profile:
    p = te_profile()
    _check(_lib.te_last_profile(H.handle, ctypes.byref(p)))
    return p


def te_spmv(H: Hamiltonian, x, y=None, stream=None):
    """y = H x and x^H y; returns (y, complex)."""
    import torch
    px = _dev_c128(x, "x", H.dim)
    if y is None:
        y = torch.empty_like(x)
    py = _dev_c128(y, "y", H.dim)
    d = te_c128()
    _check(_lib.te_spmv(H.handle, px, py, ctypes.byref(d), _stream(stream)))
    return y, complex(d.re, d.im)


def te_arnoldi(H: Hamiltonian, u, m: int, tol_rate: float, stream=None):
    """Krylov basis of u: returns (V [k, dim] tensor view, alpha[k], beta[k], k)."""
    import torch
    pu = _dev_c128(u, "u", H.dim)
    mm = min(m, H.dim)
    V = torch.empty((mm, H.dim), dtype=torch.complex128, device=u.device)
    alpha = np.zeros(mm)
    beta = np.zeros(mm)
    k = _I()
    _check(_lib.te_arnoldi(H.handle, pu, int(m), float(tol_rate), ctypes.c_void_p(V.data_ptr()),
                           alpha.ctypes.data_as(_PD), beta.ctypes.data_as(_PD), ctypes.byref(k), _stream(stream)))
    kk = k.value
    return V[:kk], alpha[:kk], beta[:kk], kk


def te_tridiag_eig(alpha, beta, stream=None):
    """Eigen-decomposition of the tridiagonal (alpha, beta): returns (lambda[k], Q[k, k])."""
    a, pa = _f64(alpha)
    k = a.size
    b, pb = _f64(beta if k > 1 else np.zeros(1))
    lam = np.zeros(k)
    Q = np.zeros(k * k)
    _check(_lib.te_tridiag_eig(k, pa, pb, lam.ctypes.data_as(_PD), Q.ctypes.data_as(_PD), _stream(stream)))
    return lam, Q.reshape(k, k).T.copy()  # C layout is column-major


def te_error_integral(lam, coef, h, a, b, options=None, stream=None):
    """Device tanh-sinh integral of h |sum coef_n exp(-i lam_n tau)| over [a, b]: (value, level, converged)."""
    l_, pl = _f64(lam)
    c_, pc = _f64(coef)
    val = _D()
    lev = _I()
    conv = _I()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.te_error_integral(l_.size, pl, pc, float(h), float(a), float(b), opt, ctypes.byref(val),
                                  ctypes.byref(lev), ctypes.byref(conv), _stream(stream)))
    return val.value, lev.value, bool(conv.value)


def te_step_search(alpha, beta, h, tol_rate, t_rem, first, tau_prev, breakdown, options=None, stream=None):
    """Step-size search of one restart: returns (tau, err, omega[k] complex, warnings)."""
    a, pa = _f64(alpha)
    k = a.size
    b, pb = _f64(beta if k > 1 else np.zeros(1))
    tau, err = _D(), _D()
    om = (te_c128 * k)()
    warn = ctypes.c_uint32()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.te_step_search(k, pa, pb, float(h), float(tol_rate), float(t_rem), int(bool(first)),
                               float(tau_prev), int(bool(breakdown)), opt, ctypes.byref(tau), ctypes.byref(err),
                               om, ctypes.byref(warn), _stream(stream)))
    omega = np.array([complex(z.re, z.im) for z in om])
    return tau.value, err.value, omega, warn.value


def te_job_footprint(dim: int, m: int) -> int:
    return int(_lib.te_job_footprint(int(dim), int(m)))


def te_engine_default_config(**overrides) -> te_engine_config:
    c = te_engine_config()
    _lib.te_engine_default_config(ctypes.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def _engine_config(m, max_jobs, hbm_budget, shape, update_rows_per_thread, flags, options, rows_per_thread=0):
    c = te_engine_default_config()
    c.m = int(m)
    c.max_jobs = int(max_jobs)
    c.hbm_budget = int(hbm_budget)
    if shape is not None:
        c.lanes_per_row, c.nnz_per_lane = int(shape[0]), int(shape[1])
    c.rows_per_thread = int(rows_per_thread)
    c.update_rows_per_thread = int(update_rows_per_thread)
    c.flags = int(flags)
    if options is not None:
        c.opt = options
    return c


class Engine:
    """te_engine_*: continuous batching of evolve jobs.  Keeps the tensors of each job alive
    until it is done; `submit` returns the job id."""

    def __init__(self, hbm_budget, m=40, max_jobs=1024, shape=None, update_rows_per_thread=0, threaded=True,
                 profile=False, options=None, stream=None, rows_per_thread=0, lane_rows=0, lane_jobs=0):
        flags = (TE_ENGINE_THREADED if threaded else 0) | (TE_ENGINE_PROFILE if profile else 0)
        cfg = _engine_config(m, max_jobs, hbm_budget, shape, update_rows_per_thread, flags, options,
                             rows_per_thread)
        cfg.lane_rows = int(lane_rows)
        cfg.lane_jobs = int(lane_jobs)
        self._e = _P()
        st = ctypes.c_void_p(0) if stream is None else _stream(stream)
        _check(_lib.te_engine_create(ctypes.byref(self._e), ctypes.byref(cfg), st))
        self._keep = {}

    def submit(self, H: Hamiltonian, v0, t: float, tol: float, out=None) -> int:
        import torch
        p0 = _dev_c128(v0, "v0", H.dim)
        if out is None:
            out = torch.empty_like(v0)
        p1 = _dev_c128(out, "out", H.dim)
        jid = _I64()
        _check(_lib.te_engine_submit(self._e, H.handle, p0, p1, float(t), float(tol), ctypes.byref(jid)))
        self._keep[jid.value] = (H, v0, out)
        return jid.value

    def output(self, job: int):
        return self._keep[job][2]

    def poll(self, job: int):
        info, res = te_job_info(), te_result()
        _check(_lib.te_engine_poll(self._e, int(job), ctypes.byref(info), ctypes.byref(res)))
        return info, res

    def wait(self, job: int = -1, timeout: float = -1.0):
        _check(_lib.te_engine_wait(self._e, int(job), float(timeout)))

    def stats(self) -> te_engine_stats:
        s = te_engine_stats()
        _check(_lib.te_engine_get_stats(self._e, ctypes.byref(s)))
        return s

    def destroy(self):
        if self._e is not None and self._e.value:
            _check(_lib.te_engine_destroy(self._e))
        self._e = None
        self._keep = {}

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def te_batch_run(groups, m=40, hbm_budget=0, max_jobs=0, shape=None, update_rows_per_thread=0, profile=False,
                 options=None, stream=None, rows_per_thread=0):
    """te_batch_create / add / launch / result / info / destroy over `groups`, a list of
    (Hamiltonian, [v0 tensors], t, tol).  Returns (outputs per group, [(te_result, status,
    te_job_info)] in submission order, te_engine_stats)."""
    import torch
    flags = TE_ENGINE_PROFILE if profile else 0
    cfg = _engine_config(m, max_jobs, 0, shape, update_rows_per_thread, flags, options, rows_per_thread)
    b = _P()
    st = ctypes.c_void_p(0) if stream is None else _stream(stream)
    _check(_lib.te_batch_create(ctypes.byref(b), ctypes.byref(cfg), st))
    outs = []
    try:
        n_total = 0
        for H, vs, t, tol in groups:
            o = [torch.empty_like(v) for v in vs]
            pv = (_P * len(vs))(*[_dev_c128(v, "v0", H.dim).value for v in vs])
            po = (_P * len(vs))(*[_dev_c128(x, "out", H.dim).value for x in o])
            first = _I()
            _check(_lib.te_batch_add(b, H.handle, len(vs), pv, po, float(t), float(tol), ctypes.byref(first)))
            outs.append(o)
            n_total += len(vs)
        stats = te_engine_stats()
        _check(_lib.te_batch_launch(b, int(hbm_budget), ctypes.byref(stats)))
        results = []
        for i in range(n_total):
            r, s, info = te_result(), _I(), te_job_info()
            _check(_lib.te_batch_result(b, i, ctypes.byref(r), ctypes.byref(s)))
            _check(_lib.te_batch_info(b, i, ctypes.byref(info)))
            results.append((r, s.value, info))
    finally:
        _lib.te_batch_destroy(b)
    return outs, results, stats


def exported_symbols():
    """Names of the C functions this binding wraps (all declared in include/te.h)."""
    return sorted(_SIGS)
