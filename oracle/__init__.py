"""ctypes binding of the sequential CPU oracle (oracle/amg_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, ENOTCONV, EBREAKDOWN, ENOTFINITE, ESTALL, ESINGULAR = range(8)

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class Params(C.Structure):
    _fields_ = [("passes_per_level", C.c_int32), ("max_coarse_rows", C.c_int32), ("max_levels", C.c_int32),
                ("max_dense_rows", C.c_int32), ("omega", C.c_double), ("pre", C.c_int32), ("post", C.c_int32),
                ("stall_ratio", C.c_double), ("hem", C.c_int32), ("alternate", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_res", C.c_double), ("true_rel_res", C.c_double),
                ("status", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
                os.path.join(_HERE, "amg_oracle.c")):
            from . import build as _b

            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_hem_pass.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p]
        L.oracle_hem_pass_desc.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p]
        L.oracle_ehem_pass.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p]
        L.oracle_number.argtypes = [C.c_int32, _i32p, _i32p]
        L.oracle_number.restype = C.c_int32
        L.oracle_rap_nnz.argtypes = [C.c_int32, _i32p, _i32p, _i32p, C.c_int32]
        L.oracle_rap_nnz.restype = C.c_int64
        L.oracle_rap.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p, C.c_int32, _i32p, _i32p, _f64p]
        L.oracle_spmv.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_spmv.restype = None
        L.oracle_lu_factor.argtypes = [C.c_int32, _f64p, _i32p]
        L.oracle_lu_solve.argtypes = [C.c_int32, _f64p, _i32p, _f64p, _f64p]
        L.oracle_lu_solve.restype = None
        L.oracle_params_default.argtypes = [C.POINTER(Params)]
        L.oracle_params_default.restype = None
        L.oracle_setup.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.POINTER(Params), C.POINTER(C.c_int32)]
        L.oracle_setup.restype = C.c_void_p
        L.oracle_nlevels.argtypes = [C.c_void_p]
        L.oracle_nlevels.restype = C.c_int32
        L.oracle_level_size.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.oracle_export_level.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_destroy.restype = None
        L.oracle_vcycle.argtypes = [C.c_void_p, _f64p, _f64p]
        L.oracle_krylov.argtypes = [C.c_void_p, C.c_int32, _f64p, _f64p, C.c_double, C.c_int32, C.c_int32,
                                    C.c_int32, C.POINTER(Info)]
        _lib = L
    return _lib


def _csr_args(a):
    return (int(a.n), np.ascontiguousarray(a.row_ptr, dtype=np.int32), np.ascontiguousarray(a.col, dtype=np.int32),
            np.ascontiguousarray(a.val, dtype=np.float64))


# ---- single steps -----------------------------------------------------------

def hem_pass(a) -> np.ndarray:
    """Algorithm 2 matching: mate[i] = partner or -1."""
    n, rp, ci, v = _csr_args(a)
    mate = np.empty(n, dtype=np.int32)
    lib().oracle_hem_pass(n, rp, ci, v, mate)
    return mate


def hem_pass_desc(a) -> np.ndarray:
    """Algorithm 2 matching from the last index: mate[i] = partner or -1."""
    n, rp, ci, v = _csr_args(a)
    mate = np.empty(n, dtype=np.int32)
    if lib().oracle_hem_pass_desc(n, rp, ci, v, mate) != 0:
        raise MemoryError("oracle_hem_pass_desc")
    return mate


def ehem_pass(a) -> np.ndarray:
    """Algorithm 3 matching (edge list sorted by weight): mate[i] = partner or -1."""
    n, rp, ci, v = _csr_args(a)
    mate = np.empty(n, dtype=np.int32)
    if lib().oracle_ehem_pass(n, rp, ci, v, mate) != 0:
        raise MemoryError("oracle_ehem_pass")
    return mate


def number(mate: np.ndarray):
    """Coarse ids in Algorithm 2's counter order: (agg, n_c)."""
    mate = np.ascontiguousarray(mate, dtype=np.int32)
    agg = np.empty(mate.size, dtype=np.int32)
    nc = lib().oracle_number(mate.size, mate, agg)
    return agg, int(nc)


def rap(a, agg: np.ndarray, nc: int):
    """Galerkin product P^T A P for the 0/1 prolongation of agg, as (row_ptr, col, val)."""
    n, rp, ci, v = _csr_args(a)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    nnz = lib().oracle_rap_nnz(n, rp, ci, agg, nc)
    crp = np.empty(nc + 1, dtype=np.int32)
    cci = np.empty(max(nnz, 1), dtype=np.int32)
    cv = np.empty(max(nnz, 1), dtype=np.float64)
    st = lib().oracle_rap(n, rp, ci, v, agg, nc, crp, cci, cv)
    assert st == OK
    return crp, cci[:nnz], cv[:nnz]


def spmv(a, x: np.ndarray) -> np.ndarray:
    n, rp, ci, v = _csr_args(a)
    y = np.empty(n)
    lib().oracle_spmv(n, rp, ci, v, np.ascontiguousarray(x, dtype=np.float64), y)
    return y


def lu_factor(a: np.ndarray):
    m = np.array(a, dtype=np.float64, order="C", copy=True)
    piv = np.empty(m.shape[0], dtype=np.int32)
    st = lib().oracle_lu_factor(m.shape[0], m, piv)
    return m, piv, st


def lu_solve(lu: np.ndarray, piv: np.ndarray, b: np.ndarray) -> np.ndarray:
    x = np.empty(lu.shape[0])
    lib().oracle_lu_solve(lu.shape[0], np.ascontiguousarray(lu), np.ascontiguousarray(piv, dtype=np.int32),
                          np.ascontiguousarray(b, dtype=np.float64), x)
    return x


# ---- hierarchy and solvers --------------------------------------------------

def default_params(**kw) -> Params:
    p = Params()
    lib().oracle_params_default(C.byref(p))
    for k, val in kw.items():
        setattr(p, k, val)
    return p


@dataclass
class Level:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    agg: np.ndarray | None


class Hierarchy:
    """Oracle AMG hierarchy (Section 3 setup phase); owns its C handle."""

    def __init__(self, a, params: Params | None = None, **kw):
        n, rp, ci, v = _csr_args(a)
        self.n = n
        p = params if params is not None else default_params(**kw)
        st = C.c_int32(0)
        self._h = lib().oracle_setup(n, rp, ci, v, C.byref(p), C.byref(st))
        self.status = st.value
        if not self._h:
            raise OracleError(self.status)

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def nlevels(self) -> int:
        return int(lib().oracle_nlevels(self._h))

    def level(self, k: int) -> Level:
        n = C.c_int32()
        nnz = C.c_int64()
        assert lib().oracle_level_size(self._h, k, C.byref(n), C.byref(nnz)) == OK
        rp = np.empty(n.value + 1, dtype=np.int32)
        ci = np.empty(max(nnz.value, 1), dtype=np.int32)
        v = np.empty(max(nnz.value, 1), dtype=np.float64)
        last = k == self.nlevels - 1
        agg = None if last else np.empty(n.value, dtype=np.int32)
        lib().oracle_export_level(self._h, k, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                  None if agg is None else agg.ctypes.data)
        return Level(n.value, rp, ci[:nnz.value], v[:nnz.value], agg)

    def vcycle(self, f: np.ndarray) -> np.ndarray:
        z = np.empty(self.n)
        lib().oracle_vcycle(self._h, np.ascontiguousarray(f, dtype=np.float64), z)
        return z

    def solve(self, b, x0=None, method: str = "pcg", rtol: float = 1e-8, maxit: int = 1000,
              true_res_period: int = 50, precond: bool = True):
        """Returns (x, info dict)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        info = Info()
        m = {"pcg": 0, "bicgstab": 1, "stationary": 2}[method]
        st = lib().oracle_krylov(self._h, m, np.ascontiguousarray(b, dtype=np.float64), x, rtol, maxit,
                                 true_res_period, int(precond), C.byref(info))
        return x, dict(status=int(st), iters=info.iters, rel_res=info.rel_res, true_rel_res=info.true_rel_res)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status
