"""Seeded synthetic inputs shared by the oracle runs and the GPU runs.

Draws index tuples, observed values (random low-rank ground truth plus
Gaussian noise), starting factors, column orders, held-out masks and fold-in
request streams.  Holds none of the factorisation method's arithmetic.

The paper's own synthetic tensors come from a generator it only cites, and
its real tensors are not available; the workloads below are synthetic stand-ins
with the shapes of the paper's S2 (3-way, 1M per mode, 100M entries, K = 100)
and a scaled S4 (5-way, K = 1000), see Table 5 of arXiv:1410.5209.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

# seeds per purpose
SEED_DATA, SEED_INIT, SEED_ORDER, SEED_TEST, SEED_REQ = 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, u64, i64, f64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        ci = ctypes.c_int
        L.synth_draw.argtypes = [u64, u64, u64]
        L.synth_draw.restype = u64
        L.synth_permutation.argtypes = [u64, u64, i64, P]
        L.synth_tuples.argtypes = [u64, ci, P, i64, ci, f64, ci, P, i64]
        L.synth_tuples.restype = i64
        L.synth_values.argtypes = [u64, ci, P, i64, P, ci, ci, f64, P]
        L.synth_values.restype = ci
        L.synth_factor.argtypes = [u64, ci, i64, ci, ci, P]
        L.synth_mask.argtypes = [u64, u64, i64, f64, P]
        L.synth_zipf_ints.argtypes = [u64, u64, i64, f64, i64, P]
        L.synth_zipf_ints.restype = ci
        L.synth_uniform_ints.argtypes = [u64, u64, i64, i64, P]
        L.synth_exponential.argtypes = [u64, u64, i64, f64, P]
        L.synth_request_values.argtypes = [u64, ci, P, ci, u64, i64, P, P, f64, P]
        L.synth_request_values.restype = ci
        L.synth_set_threads.argtypes = [ci]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(t: int) -> None:
    lib().synth_set_threads(int(t))


# ---------------------------------------------------------------------------
# primitive draws

def tuples(seed, dims, ndraw, dist="uniform", zipf_s=1.0, dedupe="distinct"):
    dims_a = np.asarray(dims, dtype=np.int64)
    N = len(dims)
    out = np.empty((max(int(ndraw), 1), N), dtype=np.int32)
    dd = {"none": 0, "drop": 1, "distinct": 2}[dedupe]
    n = lib().synth_tuples(seed, N, _p(dims_a), int(ndraw), 1 if dist == "zipf" else 0,
                           float(zipf_s), dd, _p(out), int(out.shape[0]))
    if n < 0:
        raise RuntimeError("synth_tuples failed")
    return out[:n]


def values(seed, dims, idx, R, scale, sigma):
    dims_a = np.asarray(dims, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.empty(max(idx.shape[0], 1), dtype=np.float64)
    if lib().synth_values(seed, len(dims), _p(dims_a), idx.shape[0], _p(idx), int(R),
                          int(scale), float(sigma), _p(out)) != 0:
        raise RuntimeError("synth_values failed")
    return out[: idx.shape[0]]


def factor(seed, n, I, K, zero=False):
    out = np.empty((int(I), int(K)), dtype=np.float64)
    lib().synth_factor(seed, int(n), int(I), int(K), 1 if zero else 0, _p(out))
    return out


def factors(seed, dims, K, first_zero=True):
    """Starting factors U(0,1)/sqrt(K); the first one zero (Section 3.1)."""
    return [factor(seed, n, I, K, zero=(first_zero and n == 0)) for n, I in enumerate(dims)]


def permutation(seed, stream, n):
    out = np.empty(int(n), dtype=np.int32)
    lib().synth_permutation(seed, stream, int(n), _p(out))
    return out


def column_order(seed, sweep, K):
    """A random column order for one sweep (columns chosen without replacement)."""
    return permutation(seed, 1000 + int(sweep), K)


def mask(seed, stream, n, p):
    out = np.empty(max(int(n), 1), dtype=np.uint8)
    lib().synth_mask(seed, stream, int(n), float(p), _p(out))
    return out[: int(n)].astype(bool)


def zipf_ints(seed, stream, count, s, hi):
    out = np.empty(max(int(count), 1), dtype=np.int32)
    if lib().synth_zipf_ints(seed, stream, int(count), float(s), int(hi), _p(out)) != 0:
        raise RuntimeError("synth_zipf_ints failed")
    return out[: int(count)]


def uniform_ints(seed, stream, count, n):
    out = np.empty(max(int(count), 1), dtype=np.int32)
    lib().synth_uniform_ints(seed, stream, int(count), int(n), _p(out))
    return out[: int(count)]


def exponential(seed, stream, count, rate):
    out = np.empty(max(int(count), 1), dtype=np.float64)
    lib().synth_exponential(seed, stream, int(count), float(rate), _p(out))
    return out[: int(count)]


# ---------------------------------------------------------------------------
# workloads

@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    I: int
    nnz: int            # number of draws (realised count may be lower with "drop")
    dist: str           # "uniform" | "zipf"
    zipf_s: float
    dedupe: str         # "distinct" | "drop" | "none"
    R: int              # ground-truth rank
    scale: int          # 0: x = v + noise; 1: x = 1 + 4 v / R + noise
    sigma: float
    K: int
    lam: float
    C: int
    T_in: int
    sweeps: int
    prec: str           # "f64" | "f32" | "bf16"
    test_frac: float = 0.0
    shape: tuple = ()   # mode lengths when they differ (else N modes of length I)

    @property
    def dims(self):
        return [int(d) for d in self.shape] if self.shape else [self.I] * self.N

    def replica(self, I, nnz, K=None, C=None, name=None):
        """Same recipe at a reduced size (for the oracle): every mode length
        scaled by I / self.I (at least 1), the entries to nnz."""
        f = I / self.I
        shape = tuple(max(1, int(round(d * f))) for d in self.shape) if self.shape else ()
        return replace(self, I=int(I), nnz=int(nnz), K=int(K or self.K), C=int(C or self.C),
                       shape=shape, name=name or f"{self.name}@I{I}_nnz{nnz}")


WORKLOADS = {
    # CDTF, FP64, 3-way 1000^3, 1e5 distinct uniform entries, rank-10 truth
    "cdtf-3way-1k-fp64": Workload("cdtf-3way-1k-fp64", 3, 1000, 100_000, "uniform", 0.0,
                                  "distinct", 10, 0, 0.1, 10, 0.1, 1, 1, 10, "f64"),
    # SALS C=10, FP32, 3-way 1M^3, 1e8 uniform entries (the paper's S2 shape)
    "sals-3way-1m-fp32": Workload("sals-3way-1m-fp32", 3, 1_000_000, 100_000_000, "uniform", 0.0,
                                  "distinct", 20, 1, 0.25, 100, 1.0, 10, 2, 10, "f32"),
    # SALS, FP32, 5-way 1M^5, 5e8 Zipf(1.0) draws, K = 1000 (scaled S4 shape)
    "sals-5way-zipf-fp32": Workload("sals-5way-zipf-fp32", 5, 1_000_000, 500_000_000, "zipf", 1.0,
                                    "drop", 20, 0, 0.25, 1000, 1.0, 20, 1, 1, "f32"),
    # the 5-way workload with BF16 factor storage (FP32 arithmetic)
    "sals-5way-zipf-bf16": Workload("sals-5way-zipf-bf16", 5, 1_000_000, 500_000_000, "zipf", 1.0,
                                    "drop", 20, 0, 0.25, 1000, 1.0, 20, 1, 1, "bf16"),
    # the 3-way SALS workload with BF16 factors and a 1% held-out test split
    "sals-3way-1m-bf16": Workload("sals-3way-1m-bf16", 3, 1_000_000, 100_000_000, "uniform", 0.0,
                                  "distinct", 20, 1, 0.25, 100, 1.0, 10, 2, 10, "bf16", 0.01),
    # shape-only stand-ins for the paper's real tensors (Table 4): the mode
    # lengths, entry counts, K and lambda of its Netflix_3 and Yahoo-music_4
    # runs, with uniform distinct indices and rating-like values in [1, 5]
    # (rank-20 truth + N(0, 0.25^2)); none of the datasets' content
    "netflix3-shape-fp32": Workload("netflix3-shape-fp32", 3, 2_649_429, 99_072_112, "uniform", 0.0,
                                    "distinct", 20, 1, 0.25, 40, 0.02, 10, 1, 3, "f32", 0.0,
                                    (2_649_429, 17_770, 74)),
    "yahoo4-shape-fp32": Workload("yahoo4-shape-fp32", 4, 1_000_990, 252_800_275, "uniform", 0.0,
                                  "distinct", 20, 1, 0.25, 80, 1.0, 10, 1, 3, "f32", 0.0,
                                  (1_000_990, 624_961, 133, 24)),
}


def make_tensor(w: Workload, seed=SEED_DATA):
    """Index tuples (nnz x N int32) and values (nnz float64) of a workload.

    With test_frac > 0 also returns the held-out split: (idx, x, idx_test, x_test)."""
    dims = w.dims
    idx = tuples(seed, dims, w.nnz, w.dist, w.zipf_s, w.dedupe)
    x = values(seed, dims, idx, w.R, w.scale, w.sigma)
    if w.test_frac > 0:
        m = mask(SEED_TEST, 7, idx.shape[0], w.test_frac)
        return idx[~m], x[~m], idx[m], x[m]
    return idx, x


def make_requests(dims, R, nreq, seed=SEED_REQ, data_seed=SEED_DATA, zipf_s=1.1, max_m=5000,
                  sigma=0.25):
    """Fold-in requests (new mode-0 rows): sizes Zipf(zipf_s) on [1, max_m],
    other-mode indices uniform, values from the training ground truth."""
    N = len(dims)
    sizes = zipf_ints(seed, 500, nreq, zipf_s, max_m).astype(np.int64)
    ptr = np.zeros(nreq + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    total = int(ptr[-1])
    oidx = np.empty((total, N - 1), dtype=np.int32)
    for t in range(N - 1):
        oidx[:, t] = uniform_ints(seed, 510 + t, total, dims[t + 1])
    vals = np.empty(max(total, 1), dtype=np.float64)
    dims_a = np.asarray(dims, dtype=np.int64)
    if lib().synth_request_values(data_seed, N, _p(dims_a), int(R), seed, int(nreq), _p(ptr),
                                  _p(oidx), float(sigma), _p(vals)) != 0:
        raise RuntimeError("synth_request_values failed")
    return ptr, oidx, vals[:total]
