"""Convenience wrapper over the C ABI: uploads host inputs with torch (device
memory only), holds the context and forwards every call to the HIP library."""
from __future__ import annotations

import numpy as np

from . import tf


class SparseCP:
    """One SALS/CDTF model state on the current GPU (see include/tf.h)."""

    def __init__(self, dims, idx, vals, K, lam, precision="f32", reg_mode=0,
                 first_factor_zero=True, strategy=tf.TF_STRATEGY_SKEW, seed=2, stream=None,
                 lane_nnz=2, split_threshold=4096, chunk_nnz=2048, resid_share=tf.TF_RESID_AUTO,
                 col_order=tf.TF_ORDER_FIXED, mem_budget=0, torch_alloc=False, graph=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("SparseCP needs a HIP GPU")
        self._hooks = None
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.K = int(K)
        self.lam = float(lam)
        dev = torch.device("cuda")
        d_idx = idx if isinstance(idx, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(idx, dtype=np.int32))
        d_vals = vals if isinstance(vals, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(vals, dtype=np.float64))
        d_idx = d_idx.to(dev, dtype=torch.int32).contiguous()
        d_vals = d_vals.to(dev, dtype=torch.float64).contiguous()
        self.nnz = int(d_vals.shape[0])
        opt = tf.tf_default_options(precision=precision, reg_mode=int(reg_mode),
                                    first_factor_zero=1 if first_factor_zero else 0,
                                    strategy=int(strategy), seed=int(seed), stream=stream,
                                    lane_nnz=int(lane_nnz), split_threshold=int(split_threshold),
                                    chunk_nnz=int(chunk_nnz), resid_share=int(resid_share),
                                    col_order=int(col_order), mem_budget=int(mem_budget),
                                    graph=1 if graph else 0)
        if torch_alloc:
            # the library's device memory comes from torch's caching allocator
            dev_index = torch.cuda.current_device()

            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev_index, stream or None)
                except Exception:  # out of memory: the library reports TF_E_NOMEM
                    return None

            def _free(ptr, nbytes, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._hooks = (tf.ALLOC_FN(_alloc), tf.FREE_FN(_free))
            opt.dev_alloc, opt.dev_free = self._hooks
        self.ctx = tf.tf_init(self.dims, d_idx, d_vals, self.K, self.lam, opt)
        del d_idx, d_vals  # the library keeps its own copies

    def close(self):
        if getattr(self, "ctx", None) is not None:
            tf.tf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def sweep(self, C, T_in=1):
        tf.tf_sweep(self.ctx, C, T_in)

    def split(self, cols, T_in=1):
        tf.tf_split(self.ctx, cols, T_in)

    def set_col_order(self, order):
        tf.tf_set_col_order(self.ctx, order)

    def col_order(self):
        return tf.tf_get_col_order(self.ctx, self.K)

    def loss(self):
        return tf.tf_loss(self.ctx)

    def predict(self, q):
        import torch
        q = torch.as_tensor(np.ascontiguousarray(q, dtype=np.int32)).cuda()
        out = torch.empty(q.shape[0], dtype=torch.float64, device="cuda")
        tf.tf_predict(self.ctx, q, out)
        return out.cpu().numpy()

    def factor(self, n):
        return tf.tf_get_factor(self.ctx, n, self.dims[n], self.K)

    def factor_block(self, n, rows=None, cols=None):
        return tf.tf_get_factor_block(self.ctx, n, self.dims[n], self.K, rows, cols)

    def factors(self):
        return [self.factor(n) for n in range(self.N)]

    def set_factor(self, n, A):
        tf.tf_set_factor(self.ctx, n, A)

    def set_factors(self, As, resync=True):
        for n, A in enumerate(As):
            self.set_factor(n, A)
        if resync:
            self.resync()

    def resync(self):
        tf.tf_resync(self.ctx)

    def residual(self):
        return tf.tf_get_residual(self.ctx, self.nnz)

    def csr(self, n):
        return tf.tf_get_csr(self.ctx, n, self.dims[n], self.nnz)

    def autotune(self, T_in, cands, tune_tiles=True):
        return tf.tf_autotune(self.ctx, T_in, cands, tune_tiles)

    def profile(self, enable=True):
        tf.tf_profile(self.ctx, enable)

    def profile_read(self):
        return tf.tf_profile_read(self.ctx)
