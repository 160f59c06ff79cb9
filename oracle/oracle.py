"""Python wrapper of the FP64 CPU oracle (``tf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
The C source states, function by function, which definition, equation or
algorithm of Shin & Kang (arXiv:1410.5209) it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID, E_NOMEM, E_NUMERIC = 0, 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP for the row loop only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall",
            _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        L.or_create.argtypes = [ctypes.c_int, P, i64, P, P, ctypes.c_int, f64, ctypes.c_int,
                                ctypes.POINTER(P)]
        L.or_destroy.argtypes = [P]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_set_factor.argtypes = [P, ctypes.c_int, P]
        L.or_get_factor.argtypes = [P, ctypes.c_int, P]
        L.or_get_csr.argtypes = [P, ctypes.c_int, P, P]
        L.or_get_residual.argtypes = [P, P]
        L.or_set_residual.argtypes = [P, P]
        L.or_resync.argtypes = [P]
        L.or_split.argtypes = [P, ctypes.c_int, P, ctypes.c_int]
        L.or_sweep.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        L.or_row_update.argtypes = [P, ctypes.c_int, i64, ctypes.c_int, P, P]
        L.or_bad_row.argtypes = [P]
        L.or_bad_row.restype = i64
        L.or_bad_mode.argtypes = [P]
        L.or_loss.argtypes = [P, ctypes.POINTER(f64), ctypes.POINTER(f64)]
        L.or_predict.argtypes = [P, i64, P, P]
        L.or_foldin_full.argtypes = [P, ctypes.c_int, i64, P, P, P]
        L.or_foldin_cdtf.argtypes = [P, ctypes.c_int, i64, P, P, ctypes.c_int, P]
        L.or_splitmix64.argtypes = [u64, u64]
        L.or_splitmix64.restype = u64
        L.or_init_factors.argtypes = [P, u64, ctypes.c_int]
        L.or_column_order.argtypes = [u64, i64, ctypes.c_int, P]
        L.or_column_order.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(t: int) -> None:
    lib().or_set_threads(int(t))


def get_threads() -> int:
    return int(lib().or_get_threads())


def splitmix64(seed: int, t: int) -> int:
    return int(lib().or_splitmix64(seed, t))


def column_order(seed: int, t: int, K: int) -> np.ndarray:
    """The random column order of sweep t (or_column_order)."""
    out = np.empty(int(K), dtype=np.int32)
    lib().or_column_order(int(seed), int(t), int(K), _p(out))
    return out


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle status {code} {msg}")
        self.code = code


class Oracle:
    """FP64 SALS/CDTF state: factors, residual (input order) and mode CSRs."""

    def __init__(self, dims, idx, vals, K, lam, reg_mode=0):
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.K = int(K)
        self.lam = float(lam)
        self.reg_mode = int(reg_mode)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, self.N)
        vals = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
        self.nnz = int(vals.shape[0])
        d = np.asarray(self.dims, dtype=np.int64)
        h = ctypes.c_void_p()
        rc = lib().or_create(self.N, _p(d), self.nnz, _p(idx), _p(vals), self.K, self.lam,
                             self.reg_mode, ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_destroy(h)
            self._h = None

    def set_factor(self, n, A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (self.dims[n], self.K)
        lib().or_set_factor(self._h, n, _p(A))

    def get_factor(self, n):
        A = np.empty((self.dims[n], self.K), dtype=np.float64)
        lib().or_get_factor(self._h, n, _p(A))
        return A

    def factors(self):
        return [self.get_factor(n) for n in range(self.N)]

    def get_csr(self, n):
        rp = np.empty(self.dims[n] + 1, dtype=np.int64)
        pm = np.empty(max(self.nnz, 1), dtype=np.int32)
        lib().or_get_csr(self._h, n, _p(rp), _p(pm))
        return rp, pm[: self.nnz]

    def residual(self):
        r = np.empty(max(self.nnz, 1), dtype=np.float64)
        lib().or_get_residual(self._h, _p(r))
        return r[: self.nnz]

    def set_residual(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().or_set_residual(self._h, _p(r))

    def resync(self):
        lib().or_resync(self._h)

    def split(self, cols, T_in=1):
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        rc = lib().or_split(self._h, int(cols.shape[0]), _p(cols), int(T_in))
        if rc != OK:
            raise OracleError(rc, f"split bad_row={lib().or_bad_row(self._h)}")

    def sweep(self, C, T_in=1, order=None):
        order = np.arange(self.K, dtype=np.int32) if order is None else \
            np.ascontiguousarray(order, dtype=np.int32)
        rc = lib().or_sweep(self._h, int(C), int(T_in), _p(order))
        if rc != OK:
            raise OracleError(rc, f"sweep bad_row={lib().or_bad_row(self._h)}")

    def row_update(self, n, i, cols):
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        a = np.empty(cols.shape[0], dtype=np.float64)
        rc = lib().or_row_update(self._h, int(n), int(i), int(cols.shape[0]), _p(cols), _p(a))
        if rc != OK:
            raise OracleError(rc, "row_update")
        return a

    def loss(self):
        l, r = ctypes.c_double(), ctypes.c_double()
        lib().or_loss(self._h, ctypes.byref(l), ctypes.byref(r))
        return l.value, r.value

    def predict(self, q):
        q = np.ascontiguousarray(q, dtype=np.int32).reshape(-1, self.N)
        out = np.empty(max(q.shape[0], 1), dtype=np.float64)
        rc = lib().or_predict(self._h, int(q.shape[0]), _p(q), _p(out))
        if rc != OK:
            raise OracleError(rc, "predict")
        return out[: q.shape[0]]

    def foldin_full(self, mode, oidx, vals):
        oidx = np.ascontiguousarray(oidx, dtype=np.int32).reshape(-1, self.N - 1)
        vals = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
        out = np.empty(self.K, dtype=np.float64)
        rc = lib().or_foldin_full(self._h, int(mode), int(vals.shape[0]), _p(oidx), _p(vals),
                                  _p(out))
        if rc != OK:
            raise OracleError(rc, "foldin_full")
        return out

    def foldin_cdtf(self, mode, oidx, vals, sweeps):
        oidx = np.ascontiguousarray(oidx, dtype=np.int32).reshape(-1, self.N - 1)
        vals = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
        out = np.empty(self.K, dtype=np.float64)
        rc = lib().or_foldin_cdtf(self._h, int(mode), int(vals.shape[0]), _p(oidx), _p(vals),
                                  int(sweeps), _p(out))
        if rc != OK:
            raise OracleError(rc, "foldin_cdtf")
        return out

    def init_factors(self, seed, first_factor_zero=True):
        lib().or_init_factors(self._h, int(seed), 1 if first_factor_zero else 0)
