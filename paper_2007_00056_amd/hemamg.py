"""Thin ctypes binding of libhemamg.so (include/hemamg.h).

Functions carry the C names and only marshal arguments: every step of the
setup and solve runs in the library's HIP kernels.  PyTorch supplies device
memory (tensor data pointers) and the stream.  Importing this module does not
touch the GPU; the first call loads the library and raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhemamg.so")

AMG_OK, AMG_EINVAL, AMG_ENOMEM, AMG_ENOTCONV, AMG_EBREAKDOWN, AMG_ENOTFINITE, AMG_ESTALL, AMG_ESINGULAR, AMG_EHIP = \
    range(9)
STATUS_NAMES = ["AMG_OK", "AMG_EINVAL", "AMG_ENOMEM", "AMG_ENOTCONV", "AMG_EBREAKDOWN", "AMG_ENOTFINITE",
                "AMG_ESTALL", "AMG_ESINGULAR", "AMG_EHIP"]
PCG, BICGSTAB, STATIONARY = 0, 1, 2
KERNEL_PROLONG_POST, KERNEL_RESID_RESTRICT, KERNEL_SPMV = 0, 1, 2

EXPORTED = ["amg_params_default", "amg_setup", "amg_destroy", "amg_vcycle", "krylov_solve", "amg_num_levels",
            "amg_level_size", "amg_export_level", "amg_setup_stats", "amg_timing_enable", "amg_timing_read",
            "amg_last_error", "amg_footprint_bytes", "amg_server_config_default", "amg_server_create",
            "amg_server_submit", "amg_server_wait", "amg_server_destroy", "amg_batch_create", "amg_batch_rows",
            "amg_batch_solve", "amg_batch_destroy", "amg_batch_levels", "amg_batch_autotune", "amg_autotune",
            "amg_batch_setup", "amg_batch_set_graphs", "krylov_solve_noalloc", "amg_cached_bytes",
            "amg_release_cached"]


class amg_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("val", C.c_void_p)]


class amg_params(C.Structure):
    _fields_ = [("passes_per_level", C.c_int32), ("max_coarse_rows", C.c_int32), ("max_levels", C.c_int32),
                ("max_dense_rows", C.c_int32), ("omega", C.c_double), ("pre", C.c_int32), ("post", C.c_int32),
                ("true_res_period", C.c_int32), ("precond_fp32", C.c_int32),
                ("stall_ratio", C.c_double), ("hem", C.c_int32),
                ("alternate", C.c_int32)]


class amg_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_res", C.c_double), ("true_rel_res", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("levels", C.c_int32), ("status", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class amg_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class amg_server_config(C.Structure):
    _fields_ = [("workers", C.c_int32), ("batch", C.c_int32), ("hbm_budget_bytes", C.c_uint64),
                ("params", amg_params), ("alloc", amg_allocator)]


class AmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libhemamg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2007_00056_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "amg_params_default": [C.POINTER(amg_params)],
            "amg_setup": [C.POINTER(amg_csr), C.POINTER(amg_params), C.POINTER(amg_allocator), vp, C.POINTER(vp)],
            "amg_destroy": [vp],
            "amg_vcycle": [vp, vp, vp, vp],
            "krylov_solve": [vp, i32, vp, vp, f64, i32, vp, C.POINTER(amg_info)],
            "krylov_solve_noalloc": [vp, i32, vp, vp, f64, i32, vp, C.POINTER(amg_info)],
            "amg_num_levels": [vp, C.POINTER(i32)],
            "amg_level_size": [vp, i32, C.POINTER(i32), C.POINTER(i64)],
            "amg_export_level": [vp, i32, vp, vp, vp, vp, vp],
            "amg_setup_stats": [vp, i32, vp, vp, vp, vp, C.POINTER(i32), C.POINTER(C.c_size_t)],
            "amg_timing_enable": [vp, i32, i32],
            "amg_timing_read": [vp, i32, C.POINTER(i64), C.POINTER(f64)],
            "amg_footprint_bytes": [i32, i64, C.POINTER(amg_params), C.POINTER(C.c_uint64)],
            "amg_cached_bytes": [C.POINTER(C.c_uint64)],
            "amg_release_cached": [],
            "amg_server_config_default": [C.POINTER(amg_server_config)],
            "amg_server_create": [C.POINTER(amg_server_config), C.POINTER(vp)],
            "amg_server_submit": [vp, C.POINTER(amg_csr), vp, vp, i32, f64, i32, vp, C.POINTER(i64)],
            "amg_server_wait": [vp, i64, C.POINTER(amg_info), C.POINTER(f64)],
            "amg_server_destroy": [vp],
            "amg_batch_create": [C.POINTER(vp), i32, C.POINTER(amg_allocator), vp, C.POINTER(vp)],
            "amg_batch_setup": [C.POINTER(amg_csr), i32, C.POINTER(amg_params), C.POINTER(amg_allocator), vp,
                                C.POINTER(vp), vp],
            "amg_batch_set_graphs": [vp, i32],
            "amg_batch_rows": [vp, vp],
            "amg_batch_solve": [vp, i32, vp, vp, f64, i32, vp, vp],
            "amg_batch_destroy": [vp],
            "amg_batch_levels": [vp, C.POINTER(i32)],
            "amg_batch_autotune": [vp, vp, vp],
            "amg_autotune": [vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.amg_last_error.argtypes = []
        L.amg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != AMG_OK:
        raise AmgError(st, lib().amg_last_error().decode())


def _stream_ptr(stream) -> int | None:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def _ptr(t) -> int:
    return t.data_ptr()


def _info_dict(st: int, info: amg_info) -> dict:
    return dict(status=st, iters=info.iters, rel_res=info.rel_res, true_rel_res=info.true_rel_res,
                setup_ms=info.setup_ms, solve_ms=info.solve_ms, levels=info.levels)


class Allocator:
    """An amg_allocator whose alloc/free are Python callables
    alloc(nbytes, stream) -> device address (0 on failure) and
    free(address, stream).  Keep the object alive while any handle, batch or
    server uses it (the C side holds its function pointers)."""

    def __init__(self, alloc, free):
        def _a(size, ctx, stream):
            try:
                return int(alloc(int(size), int(stream or 0))) or None
            except Exception:  # the library turns NULL into AMG_ENOMEM
                return None

        def _f(ptr, ctx, stream):
            free(int(ptr), int(stream or 0))

        self._a, self._f = ALLOC_FN(_a), FREE_FN(_f)
        self.c = amg_allocator(self._a, self._f, None)


class TorchAllocator(Allocator):
    """Routes device memory through PyTorch's caching allocator, so torch's
    memory statistics and limits see every byte a handle owns."""

    def __init__(self, device=None):
        import torch

        dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
        super().__init__(lambda n, st: torch.cuda.caching_allocator_alloc(n, dev, st),
                         lambda p, st: torch.cuda.caching_allocator_delete(p))


def _alloc_ref(alloc):
    return C.byref(alloc.c) if alloc is not None else None


# ---------------------------------------------------------------- C entry points

def amg_params_default(**overrides) -> amg_params:
    p = amg_params()
    _check(lib().amg_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class DeviceCSR:
    """CSR matrix in GPU memory (torch tensors) plus its amg_csr view."""

    def __init__(self, row_ptr, col_idx, val):
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val
        self.n = int(row_ptr.numel() - 1)
        self.nnz = int(col_idx.numel())
        self.c = amg_csr(self.n, self.nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val))

    @classmethod
    def from_host(cls, a, device="cuda"):
        import torch

        return cls(torch.from_numpy(np.ascontiguousarray(a.row_ptr, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(a.col, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(a.val, dtype=np.float64)).to(device))


def amg_setup(A: DeviceCSR, params: amg_params | None = None, stream=None, alloc: Allocator | None = None) -> int:
    """Returns the handle (an opaque pointer value)."""
    h = C.c_void_p()
    _check(lib().amg_setup(C.byref(A.c), C.byref(params) if params is not None else None, _alloc_ref(alloc),
                           _stream_ptr(stream), C.byref(h)))
    return h.value


def amg_destroy(h: int) -> None:
    _check(lib().amg_destroy(h))


def amg_vcycle(h: int, r, z, stream=None) -> None:
    _check(lib().amg_vcycle(h, _ptr(r), _ptr(z), _stream_ptr(stream)))


def krylov_solve(h: int, method: int, b, x, rtol: float, maxit: int, stream=None, check: bool = True) -> dict:
    info = amg_info()
    st = lib().krylov_solve(h, method, _ptr(b), _ptr(x), rtol, maxit, _stream_ptr(stream), C.byref(info))
    out = _info_dict(st, info)
    if check and st not in (AMG_OK,):
        raise AmgError(st, lib().amg_last_error().decode())
    return out


def krylov_solve_noalloc(h: int, method: int, b, x, rtol: float, maxit: int, stream=None,
                         check: bool = True) -> dict:
    """krylov_solve with the work vectors in the library's static scratch
    (no allocation during the call; level 0 of at most 2^20 rows)."""
    info = amg_info()
    st = lib().krylov_solve_noalloc(h, method, _ptr(b), _ptr(x), rtol, maxit, _stream_ptr(stream), C.byref(info))
    out = _info_dict(st, info)
    if check and st not in (AMG_OK,):
        raise AmgError(st, lib().amg_last_error().decode())
    return out


def amg_num_levels(h: int) -> int:
    n = C.c_int32()
    _check(lib().amg_num_levels(h, C.byref(n)))
    return n.value


def amg_level_size(h: int, k: int):
    n, nnz = C.c_int32(), C.c_int64()
    _check(lib().amg_level_size(h, k, C.byref(n), C.byref(nnz)))
    return n.value, nnz.value


def amg_export_level(h: int, k: int, stream=None):
    """Level k as host arrays (row_ptr, col_idx, val, agg or None)."""
    n, nnz = amg_level_size(h, k)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(max(nnz, 1), np.int32)
    v = np.empty(max(nnz, 1), np.float64)
    last = k == amg_num_levels(h) - 1
    agg = None if last else np.empty(n, np.int32)
    _check(lib().amg_export_level(h, k, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                  None if agg is None else agg.ctypes.data, _stream_ptr(stream)))
    return rp, ci[:nnz], v[:nnz], agg


def amg_setup_stats(h: int):
    """Per matching pass: rounds, GPU ms, rows and entries of the matched
    operator; and the bytes the handle owns."""
    cap = 256
    rounds = np.zeros(cap, np.int32)
    ms = np.zeros(cap, np.float64)
    pn = np.zeros(cap, np.int32)
    pz = np.zeros(cap, np.int64)
    npass = C.c_int32()
    owned = C.c_size_t()
    _check(lib().amg_setup_stats(h, cap, rounds.ctypes.data, ms.ctypes.data, pn.ctypes.data, pz.ctypes.data,
                                 C.byref(npass), C.byref(owned)))
    k = min(npass.value, cap)
    return dict(rounds=rounds[:k].tolist(), match_ms=ms[:k].tolist(), pass_n=pn[:k].tolist(), pass_nnz=pz[:k].tolist(),
                owned_bytes=owned.value)


def amg_timing_enable(h: int, kernel: int, on: bool = True) -> None:
    _check(lib().amg_timing_enable(h, kernel, int(on)))


def amg_timing_read(h: int, kernel: int):
    cnt, ms = C.c_int64(), C.c_double()
    _check(lib().amg_timing_read(h, kernel, C.byref(cnt), C.byref(ms)))
    return cnt.value, ms.value


def amg_last_error() -> str:
    return lib().amg_last_error().decode()


def amg_footprint_bytes(n: int, nnz: int, params: amg_params | None = None) -> int:
    b = C.c_uint64()
    _check(lib().amg_footprint_bytes(n, nnz, C.byref(params) if params is not None else None, C.byref(b)))
    return b.value


def amg_cached_bytes() -> int:
    """Device memory the library keeps for reuse on the current device."""
    b = C.c_uint64()
    _check(lib().amg_cached_bytes(C.byref(b)))
    return b.value


def amg_release_cached() -> None:
    """Frees the kept chunks and trims the library pool (current device)."""
    _check(lib().amg_release_cached())


def amg_server_config_default(**overrides) -> amg_server_config:
    c = amg_server_config()
    _check(lib().amg_server_config_default(C.byref(c)))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def amg_server_create(config: amg_server_config | None = None) -> int:
    h = C.c_void_p()
    _check(lib().amg_server_create(C.byref(config) if config is not None else None, C.byref(h)))
    return h.value


def amg_server_submit(s: int, A: DeviceCSR, b, x, method: int, rtol: float, maxit: int, stream=None) -> int:
    """stream: where b and x were produced (default: torch's current stream)."""
    t = C.c_int64()
    _check(lib().amg_server_submit(s, C.byref(A.c), _ptr(b), _ptr(x), method, rtol, maxit, _stream_ptr(stream),
                                   C.byref(t)))
    return t.value


def amg_server_wait(s: int, ticket: int) -> dict:
    """Waits for one request; returns its summary with the status (not raised)."""
    info = amg_info()
    lat = C.c_double()
    st = lib().amg_server_wait(s, ticket, C.byref(info), C.byref(lat))
    return dict(_info_dict(st, info), latency_ms=lat.value)


def amg_server_destroy(s: int) -> None:
    _check(lib().amg_server_destroy(s))


def amg_batch_create(handles, stream=None, alloc: Allocator | None = None) -> int:
    arr = (C.c_void_p * len(handles))(*handles)
    b = C.c_void_p()
    _check(lib().amg_batch_create(arr, len(handles), _alloc_ref(alloc), _stream_ptr(stream), C.byref(b)))
    return b.value


def amg_batch_setup(systems, params: amg_params | None = None, stream=None, alloc: Allocator | None = None):
    """Builds the hierarchies of every system together; returns (batch handle,
    per-system statuses)."""
    arr = (amg_csr * len(systems))(*[A.c for A in systems])
    st = np.zeros(len(systems), np.int32)
    b = C.c_void_p()
    _check(lib().amg_batch_setup(arr, len(systems), C.byref(params) if params is not None else None,
                                 _alloc_ref(alloc), _stream_ptr(stream), C.byref(b), st.ctypes.data))
    return b.value, st.tolist()


def amg_batch_rows(b: int, count: int) -> np.ndarray:
    off = np.empty(count + 1, np.int32)
    _check(lib().amg_batch_rows(b, off.ctypes.data))
    return off


def amg_batch_solve(b: int, method: int, rhs, x, rtol: float, maxit: int, count: int, stream=None) -> list:
    """Solves every system of the batch; returns one summary per system (the
    statuses are reported, not raised)."""
    infos = (amg_info * count)()
    lib().amg_batch_solve(b, method, _ptr(rhs), _ptr(x), rtol, maxit, _stream_ptr(stream), infos)
    return [_info_dict(i.status, i) for i in infos]


def amg_autotune(h: int, stream=None) -> list:
    """Tunes the hierarchy's V-cycle schedule in place; returns it per level."""
    out = np.zeros(amg_num_levels(h), np.int32)
    _check(lib().amg_autotune(h, _stream_ptr(stream), out.ctypes.data))
    return out.tolist()


def amg_batch_levels(b: int) -> int:
    n = C.c_int32()
    _check(lib().amg_batch_levels(b, C.byref(n)))
    return n.value


def amg_batch_autotune(b: int, stream=None) -> list:
    out = np.zeros(amg_batch_levels(b), np.int32)
    _check(lib().amg_batch_autotune(b, _stream_ptr(stream), out.ctypes.data))
    return out.tolist()


def amg_batch_destroy(b: int) -> None:
    _check(lib().amg_batch_destroy(b))


# ---------------------------------------------------------------- convenience

class Hierarchy:
    """Owns an amg_setup handle and the device matrix it borrows."""

    def __init__(self, A: DeviceCSR, params: amg_params | None = None, stream=None, alloc: Allocator | None = None,
                 **overrides):
        if params is None:
            params = amg_params_default(**overrides)
        self.A = A  # level 0 is borrowed: keep it alive
        self.params = params
        self.alloc = alloc  # its callbacks must outlive the handle
        self.h = amg_setup(A, params, stream, alloc)

    def close(self):
        if getattr(self, "h", None):
            amg_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def nlevels(self) -> int:
        return amg_num_levels(self.h)

    def level(self, k: int):
        return amg_export_level(self.h, k)

    def vcycle(self, r, z=None, stream=None):
        import torch

        z = torch.empty_like(r) if z is None else z
        amg_vcycle(self.h, r, z, stream)
        return z

    def solve(self, b, x=None, method: str = "pcg", rtol: float = 1e-8, maxit: int = 1000, stream=None,
              check: bool = True):
        import torch

        x = torch.zeros_like(b) if x is None else x
        info = krylov_solve(self.h, {"pcg": PCG, "bicgstab": BICGSTAB, "stationary": STATIONARY}[method], b, x, rtol,
                            maxit, stream, check)
        return x, info

    def stats(self):
        return amg_setup_stats(self.h)

    def autotune(self, stream=None) -> list:
        return amg_autotune(self.h, stream)


class Batch:
    """Owns a batch built from hierarchies (amg_batch_create) or set up from
    matrices (Batch.setup, amg_batch_setup)."""

    def __init__(self, hierarchies=None, stream=None, alloc: Allocator | None = None, _handle=None, _count=None):
        self.alloc = alloc
        if _handle is not None:
            self.count, self.b = _count, _handle
        else:
            self.count = len(hierarchies)
            self.b = amg_batch_create([h.h if isinstance(h, Hierarchy) else h for h in hierarchies], stream, alloc)
        self.status = [AMG_OK] * self.count
        self.offsets = amg_batch_rows(self.b, self.count)

    @classmethod
    def setup(cls, systems, params: amg_params | None = None, stream=None, alloc: Allocator | None = None,
              **overrides):
        """systems: DeviceCSR matrices (borrowed during the call only)."""
        if params is None:
            params = amg_params_default(**overrides)
        h, st = amg_batch_setup(systems, params, stream, alloc)
        bt = cls(alloc=alloc, _handle=h, _count=len(systems))
        bt.status = st
        return bt

    def close(self):
        if getattr(self, "b", None):
            amg_batch_destroy(self.b)
            self.b = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, rhs, x=None, rtol: float = 1e-8, maxit: int = 1000, stream=None, method: str = "pcg"):
        """rhs, x: device float64 vectors of offsets[-1] rows (systems one after
        another).  Returns (x, list of per-system summaries)."""
        import torch

        x = torch.zeros_like(rhs) if x is None else x
        m = {"pcg": PCG, "bicgstab": BICGSTAB}[method]
        return x, amg_batch_solve(self.b, m, rhs, x, rtol, maxit, self.count, stream)

    def autotune(self, stream=None) -> list:
        return amg_batch_autotune(self.b, stream)

    def set_graphs(self, on: bool) -> None:
        _check(lib().amg_batch_set_graphs(self.b, int(on)))
