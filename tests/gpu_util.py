"""Shared helpers of the GPU tests: build the GPU model and the oracle from the
same seeded inputs, and compare them."""
import sys

import numpy as np

import synth
from oracle import oracle as orc


def note(msg):
    """Name the case before a GPU step (a crashed box returns only the log tail)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def problem(seed, dims, nnz, K, dist="uniform", dedupe="distinct", zipf_s=1.0, R=3, scale=0,
            sigma=0.1, first_zero=True):
    idx = synth.tuples(seed, dims, nnz, dist=dist, zipf_s=zipf_s, dedupe=dedupe)
    x = synth.values(seed, dims, idx, R, scale, sigma)
    A = synth.factors(seed + 1000, dims, K, first_zero=first_zero)
    return idx, x, A


def pair(dims, idx, x, A, K, lam, precision="f64", reg_mode=0, **opts):
    """GPU model and oracle, both starting from factors A and r = x - recon."""
    from paper_1410_5209_amd.model import SparseCP
    g = SparseCP(dims, idx, x, K, lam, precision=precision, reg_mode=reg_mode, **opts)
    g.set_factors(A)
    o = orc.Oracle(dims, idx, x, K, lam, reg_mode)
    for n, An in enumerate(A):
        o.set_factor(n, An)
    o.resync()
    return g, o


def rel_max(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def recon(dims, idx, A):
    prod = np.ones((idx.shape[0], A[0].shape[1]))
    for n in range(len(dims)):
        prod = prod * A[n][idx[:, n]]
    return prod.sum(axis=1)
