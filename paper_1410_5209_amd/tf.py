"""Thin ctypes binding of the C ABI in include/tf.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device buffers are
passed as torch tensors (their data pointers); host buffers as numpy arrays.
All computation runs in the HIP library; if it is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TFSALS_LIB") or os.path.join(_HERE, "libtfsals.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "tf.h")

TF_OK, TF_E_INVALID, TF_E_NOMEM, TF_E_DEVICE, TF_E_NUMERIC, TF_E_UNSUPPORTED, TF_E_BUSY, TF_E_STATE = range(8)
TF_PREC_F64, TF_PREC_F32, TF_PREC_BF16 = 0, 1, 2
TF_STRATEGY_PLAIN, TF_STRATEGY_SKEW, TF_STRATEGY_AUTO, TF_STRATEGY_PERSISTENT = 0, 1, 2, 3
TF_RESID_AUTO, TF_RESID_OWN, TF_RESID_SHARED = 0, 1, 2
TF_ORDER_FIXED, TF_ORDER_RANDOM = 0, 1

# device memory hooks (tf_alloc_fn / tf_free_fn)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
PREC = {"f64": TF_PREC_F64, "f32": TF_PREC_F32, "bf16": TF_PREC_BF16}


class tf_options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("reg_mode", ctypes.c_int32), ("first_factor_zero", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("lane_nnz", ctypes.c_int32),
                ("split_threshold", ctypes.c_int32), ("chunk_nnz", ctypes.c_int32),
                ("resid_share", ctypes.c_int32), ("col_order", ctypes.c_int32),
                ("mem_budget", ctypes.c_size_t), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_user", ctypes.c_void_p), ("graph", ctypes.c_int32)]


class tf_kstats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("sweeps", ctypes.c_int64),
                ("first_launches", ctypes.c_int64), ("first_ms", ctypes.c_double),
                ("first_bytes", ctypes.c_double), ("graph_sweeps", ctypes.c_int64)]


class tf_plan_summary(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int64), ("split_rows", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("empty_rows", ctypes.c_int64),
                ("rows_by_lanes", ctypes.c_int64 * 7)]


class tf_serve_opts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("method", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("mem_budget", ctypes.c_int64)]


class tf_request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("h_idx", ctypes.c_void_p), ("h_vals", ctypes.c_void_p)]


class tf_req_stats(ctypes.Structure):
    _fields_ = [("latency_us", ctypes.c_double), ("queue_us", ctypes.c_double),
                ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32)]


class tf_serve_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("busy_rejects", ctypes.c_int64), ("max_queue", ctypes.c_int64),
                ("p50_us", ctypes.c_double), ("p90_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("p999_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("solves_per_s", ctypes.c_double), ("mean_batch", ctypes.c_double),
                ("failed", ctypes.c_int64)]


TF_FOLDIN_FULL, TF_FOLDIN_CDTF = 0, 1


class tf_tune_result(ctypes.Structure):
    _fields_ = [("best_C", ctypes.c_int32), ("ncand", ctypes.c_int32),
                ("cand_C", ctypes.c_int32 * 16), ("est_sweep_ms", ctypes.c_double * 16),
                ("lane_nnz", ctypes.c_int32 * 8), ("split_threshold", ctypes.c_int32 * 8),
                ("chunk_nnz", ctypes.c_int32 * 8), ("tune_ms", ctypes.c_double),
                ("persistent", ctypes.c_int32 * 8)]


class TFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tf status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libtfsals.so (built by paper_1410_5209_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.tf_default_options.argtypes = [ctypes.POINTER(tf_options)]
        L.tf_default_options.restype = None
        L.tf_init.argtypes = [ctypes.POINTER(P), i32, P, i64, P, P, i32, f64, ctypes.POINTER(tf_options)]
        L.tf_destroy.argtypes = [P]
        L.tf_destroy.restype = None
        L.tf_last_error.argtypes = [P]
        L.tf_last_error.restype = ctypes.c_char_p
        L.tf_sweep.argtypes = [P, i32, i32]
        L.tf_split.argtypes = [P, i32, P, i32]
        L.tf_set_col_order.argtypes = [P, P]
        L.tf_get_col_order.argtypes = [P, P]
        L.tf_loss.argtypes = [P, ctypes.POINTER(f64), ctypes.POINTER(f64)]
        L.tf_predict.argtypes = [P, i64, P, P]
        L.tf_get_factor.argtypes = [P, i32, P]
        L.tf_get_factor_block.argtypes = [P, i32, ctypes.c_int64, P, i32, P, P]
        L.tf_set_factor.argtypes = [P, i32, P]
        L.tf_resync.argtypes = [P]
        L.tf_get_residual.argtypes = [P, P]
        L.tf_get_csr.argtypes = [P, i32, P, P]
        L.tf_profile.argtypes = [P, i32]
        L.tf_profile_read.argtypes = [P, ctypes.POINTER(tf_kstats)]
        L.tf_plan_rows.argtypes = [P, i64, i32, i32, i32, i32, ctypes.POINTER(tf_plan_summary)]
        L.tf_foldin.argtypes = [P, i32, i32, P, P, P, i32, i32, P]
        L.tf_foldin_noalloc.argtypes = [P, i32, i32, P, P, P, i32, i32, P]
        L.tf_autotune.argtypes = [P, i32, P, i32, i32, ctypes.POINTER(tf_tune_result)]
        L.tf_serve_default_options.argtypes = [ctypes.POINTER(tf_serve_opts)]
        L.tf_serve_default_options.restype = None
        L.tf_serve_open.argtypes = [P, ctypes.POINTER(tf_serve_opts), ctypes.POINTER(P)]
        L.tf_serve_submit.argtypes = [P, ctypes.POINTER(tf_request), ctypes.POINTER(ctypes.c_uint64)]
        L.tf_serve_wait.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(tf_req_stats)]
        L.tf_serve_replay.argtypes = [P, i64, P, P, P]
        L.tf_serve_report.argtypes = [P, ctypes.POINTER(tf_serve_stats)]
        L.tf_serve_reset_stats.argtypes = [P]
        L.tf_serve_close.argtypes = [P]
        L.tf_serve_close.restype = None
        L.tf_serve_last_error.argtypes = [P]
        L.tf_serve_last_error.restype = ctypes.c_char_p
        L.tf_serve_inject_fault.argtypes = [P, ctypes.c_int32]
        L.tf_probe_gather.argtypes = [P, i64, i64, i64, ctypes.c_uint64, P, P,
                                      ctypes.POINTER(ctypes.c_double)]
        for name in ("tf_init", "tf_sweep", "tf_split", "tf_set_col_order", "tf_get_col_order",
                     "tf_loss", "tf_predict", "tf_get_factor", "tf_get_factor_block", "tf_set_factor",
                     "tf_resync",
                     "tf_get_residual", "tf_get_csr", "tf_profile", "tf_profile_read",
                     "tf_plan_rows", "tf_foldin", "tf_foldin_noalloc", "tf_serve_open", "tf_serve_submit",
                     "tf_serve_wait", "tf_serve_replay", "tf_serve_report",
                     "tf_serve_reset_stats", "tf_autotune"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _np(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, status):
    if status != TF_OK:
        raise TFError(status, lib().tf_last_error(ctx).decode())


def tf_default_options(**kw) -> tf_options:
    o = tf_options()
    lib().tf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PREC[v]
        if k == "stream" and v is not None and not isinstance(v, int):
            v = v.cuda_stream  # a torch.cuda.Stream
        setattr(o, k, v)
    return o


def tf_init(dims, d_idx, d_vals, K, lam, opt: tf_options | None = None):
    """d_idx: device int32 (nnz, N); d_vals: device float64 (nnz,). Returns ctx."""
    dims_a = np.ascontiguousarray(dims, dtype=np.int64)
    assert d_idx.is_contiguous() and d_vals.is_contiguous()
    ctx = ctypes.c_void_p()
    st = lib().tf_init(ctypes.byref(ctx), len(dims_a), _np(dims_a), int(d_vals.shape[0]),
                       _dev(d_idx), _dev(d_vals), int(K), float(lam),
                       ctypes.byref(opt) if opt is not None else None)
    _check(None, st)
    return ctx


def tf_destroy(ctx):
    lib().tf_destroy(ctx)


def tf_last_error(ctx):
    return lib().tf_last_error(ctx).decode()


def tf_sweep(ctx, C, T_in=1):
    _check(ctx, lib().tf_sweep(ctx, int(C), int(T_in)))


def tf_split(ctx, cols, T_in=1):
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    _check(ctx, lib().tf_split(ctx, int(cols.shape[0]), _np(cols), int(T_in)))


def tf_set_col_order(ctx, order):
    order = np.ascontiguousarray(order, dtype=np.int32)
    _check(ctx, lib().tf_set_col_order(ctx, _np(order)))


def tf_get_col_order(ctx, K):
    out = np.empty(int(K), dtype=np.int32)
    _check(ctx, lib().tf_get_col_order(ctx, _np(out)))
    return out


def tf_loss(ctx):
    l, r = ctypes.c_double(), ctypes.c_double()
    _check(ctx, lib().tf_loss(ctx, ctypes.byref(l), ctypes.byref(r)))
    return l.value, r.value


def tf_predict(ctx, d_idx, d_out):
    _check(ctx, lib().tf_predict(ctx, int(d_idx.shape[0]), _dev(d_idx), _dev(d_out)))


def tf_get_factor_block(ctx, n, I, K, rows=None, cols=None):
    """Rows `rows` and columns `cols` (None: all) of factor n as FP64."""
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    c = None if cols is None else np.ascontiguousarray(cols, dtype=np.int32)
    nr = int(I) if r is None else int(r.shape[0])
    nc = int(K) if c is None else int(c.shape[0])
    out = np.empty((nr, nc), dtype=np.float64)
    _check(ctx, lib().tf_get_factor_block(ctx, int(n), nr, None if r is None else _np(r), nc,
                                          None if c is None else _np(c), _np(out)))
    return out


def tf_get_factor(ctx, n, I, K):
    out = np.empty((int(I), int(K)), dtype=np.float64)
    _check(ctx, lib().tf_get_factor(ctx, int(n), _np(out)))
    return out


def tf_set_factor(ctx, n, A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    _check(ctx, lib().tf_set_factor(ctx, int(n), _np(A)))


def tf_resync(ctx):
    _check(ctx, lib().tf_resync(ctx))


def tf_get_residual(ctx, nnz):
    out = np.empty(int(nnz), dtype=np.float64)
    _check(ctx, lib().tf_get_residual(ctx, _np(out)))
    return out


def tf_get_csr(ctx, n, I, nnz):
    rp = np.empty(int(I) + 1, dtype=np.int64)
    pm = np.empty(int(nnz), dtype=np.int32)
    _check(ctx, lib().tf_get_csr(ctx, int(n), _np(rp), _np(pm)))
    return rp, pm


def tf_profile(ctx, enable=True):
    _check(ctx, lib().tf_profile(ctx, 1 if enable else 0))


def tf_profile_read(ctx) -> tf_kstats:
    s = tf_kstats()
    _check(ctx, lib().tf_profile_read(ctx, ctypes.byref(s)))
    return s


def tf_plan_rows(rowptr, strategy=TF_STRATEGY_SKEW, lane_nnz=2, split_threshold=4096,
                 chunk_nnz=2048) -> tf_plan_summary:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    s = tf_plan_summary()
    _check(None, lib().tf_plan_rows(_np(rowptr), int(rowptr.shape[0] - 1), int(strategy),
                                    int(lane_nnz), int(split_threshold), int(chunk_nnz),
                                    ctypes.byref(s)))
    return s


def tf_autotune(ctx, T_in, cands, tune_tiles=True) -> tf_tune_result:
    cands = np.ascontiguousarray(cands, dtype=np.int32)
    r = tf_tune_result()
    _check(ctx, lib().tf_autotune(ctx, int(T_in), _np(cands), int(cands.shape[0]),
                                  1 if tune_tiles else 0, ctypes.byref(r)))
    return r


def tf_foldin(ctx, mode, h_req_ptr, d_idx, d_vals, method, sweeps, d_rows):
    """h_req_ptr host int64 (nreq+1); d_idx device int32 (total, N-1); d_vals
    device float64 (total,); d_rows device float64 (nreq, K)."""
    h_req_ptr = np.ascontiguousarray(h_req_ptr, dtype=np.int64)
    nreq = int(h_req_ptr.shape[0] - 1)
    _check(ctx, lib().tf_foldin(ctx, int(mode), nreq, _np(h_req_ptr), _dev(d_idx), _dev(d_vals),
                                int(method), int(sweeps), _dev(d_rows)))


def tf_serve_default_options(**kw) -> tf_serve_opts:
    o = tf_serve_opts()
    lib().tf_serve_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def tf_serve_open(ctx, opts: tf_serve_opts | None = None):
    srv = ctypes.c_void_p()
    _check(ctx, lib().tf_serve_open(ctx, ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(srv)))
    return srv


def make_request(idx, vals):
    """A tf_request over host arrays (kept alive by the caller)."""
    r = tf_request()
    r.m = int(vals.shape[0])
    r.h_idx = idx.ctypes.data if r.m else None
    r.h_vals = vals.ctypes.data if r.m else None
    return r


def tf_serve_submit(srv, req: tf_request):
    t = ctypes.c_uint64()
    st = lib().tf_serve_submit(srv, ctypes.byref(req), ctypes.byref(t))
    if st != TF_OK:
        raise TFError(st, "tf_serve_submit")
    return t.value


def tf_serve_wait(srv, ticket, K):
    row = np.empty(int(K), dtype=np.float64)
    st = tf_req_stats()
    rc = lib().tf_serve_wait(srv, ctypes.c_uint64(ticket), _np(row), ctypes.byref(st))
    if rc != TF_OK:
        raise TFError(rc, "tf_serve_wait")
    return row, st


def tf_serve_wait_status(srv, ticket, K):
    """tf_serve_wait without raising: (status, row, stats)."""
    row = np.empty(int(K), dtype=np.float64)
    st = tf_req_stats()
    rc = lib().tf_serve_wait(srv, ctypes.c_uint64(ticket), _np(row), ctypes.byref(st))
    return int(rc), row, st


def tf_probe_gather(d_table, rows, waves, steps, seed, d_out, stream=None) -> float:
    """Milliseconds of one random-row gather launch (see include/tf.h)."""
    ms = ctypes.c_double()
    _check(None, lib().tf_probe_gather(_dev(d_table), int(rows), int(waves), int(steps),
                                       ctypes.c_uint64(seed), _dev(d_out), stream,
                                       ctypes.byref(ms)))
    return ms.value


def tf_serve_last_error(srv) -> str:
    return lib().tf_serve_last_error(srv).decode()


def tf_serve_inject_fault(srv, nbatches):
    _check(None, lib().tf_serve_inject_fault(srv, int(nbatches)))


def tf_serve_replay(srv, arrival_s, reqs):
    arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
    n = len(reqs)
    arr = (tf_request * n)(*reqs)
    tickets = np.empty(n, dtype=np.uint64)
    rc = lib().tf_serve_replay(srv, n, _np(arrival_s), ctypes.cast(arr, ctypes.c_void_p),
                               _np(tickets))
    if rc != TF_OK:
        raise TFError(rc, "tf_serve_replay")
    return tickets


def tf_serve_report(srv) -> tf_serve_stats:
    r = tf_serve_stats()
    _check(None, lib().tf_serve_report(srv, ctypes.byref(r)))
    return r


def tf_serve_reset_stats(srv):
    _check(None, lib().tf_serve_reset_stats(srv))


def tf_serve_close(srv):
    lib().tf_serve_close(srv)


def declared_symbols(header: str = HEADER):
    """Names of the functions include/tf.h declares."""
    import re
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tf_[a-z0-9_]+)\s*\(", text)))
