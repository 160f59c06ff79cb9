"""tf_foldin_noalloc (the fold-in entry point that allocates nothing) against
tf_foldin through the C ABI: the same rows bit for bit, on two calls in a row
(the second with a smaller batch, so the scratch array holds the first
call's contents when the second starts), with the model's device memory in
torch's caching allocator so that any allocation through the context would
show; a batch beyond the scratch array is refused with a message."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import note, pair, problem

pytestmark = pytest.mark.gpu


def _batch(dims, sizes, seed):
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(ptr[-1])
    oidx = np.stack([synth.uniform_ints(seed, 80 + t, total, dims[t + 1]) for t in range(2)],
                    axis=1).astype(np.int32)
    vals = synth.values(seed, dims[1:], oidx, 2, 0, 0.1)
    return ptr, oidx, vals


def _run(fn, g, ptr, oidx, vals, method):
    import torch
    from paper_1410_5209_amd import tf
    d_idx = torch.from_numpy(np.ascontiguousarray(oidx)).cuda()
    d_vals = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
    rows = torch.full((len(ptr) - 1, g.K), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    rc = fn(g.ctx, 0, len(ptr) - 1, tf._np(ptr), tf._dev(d_idx), tf._dev(d_vals), method, 3,
            tf._dev(rows))
    torch.cuda.synchronize()
    grew = torch.cuda.max_memory_allocated() - before    # peak during the call
    return rc, rows.cpu().numpy(), grew


@pytest.mark.parametrize("prec,K", [("f32", 100), ("f64", 24), ("f32", 160)])
def test_noalloc_foldin_equals_foldin_on_two_calls(prec, K):
    from paper_1410_5209_amd import tf
    dims = [500, 400, 300]
    note(f"no-alloc fold-in {prec} K={K}")
    idx, x, A = problem(90, dims, 30000, K, first_zero=False)
    g, _ = pair(dims, idx, x, A, K, 0.7, prec, torch_alloc=True)
    L = tf.lib()
    methods = [tf.TF_FOLDIN_CDTF] if K > 128 else [tf.TF_FOLDIN_FULL, tf.TF_FOLDIN_CDTF]
    for method in methods:
        for sizes, seed in (([700, 1, 0, 3000, 45, 260, 12], 5), ([9, 300, 2], 6)):
            ptr, oidx, vals = _batch(dims, sizes, seed)
            rc0, want, grew0 = _run(L.tf_foldin, g, ptr, oidx, vals, method)
            rc1, got, grew = _run(L.tf_foldin_noalloc, g, ptr, oidx, vals, method)
            assert rc0 == tf.TF_OK and rc1 == tf.TF_OK
            assert grew0 > 0                       # the measurement sees tf_foldin's workspace
            assert grew == 0                       # no allocation through the context, even briefly
            assert np.array_equal(got, want)       # same kernels, same sums: bit for bit
    g.close()


def test_noalloc_foldin_refuses_a_batch_beyond_its_scratch():
    from paper_1410_5209_amd import tf
    dims, K = [200, 3000, 3000], 100
    note("no-alloc fold-in too large")
    idx, x, A = problem(91, dims, 20000, K)
    g, _ = pair(dims, idx, x, A, K, 0.7, "f32")
    ptr, oidx, vals = _batch(dims, [5000] * 20, 7)          # 1e5 entries: ~48 MB of workspace
    rc, rows, _ = _run(tf.lib().tf_foldin_noalloc, g, ptr, oidx, vals, tf.TF_FOLDIN_FULL)
    assert rc == tf.TF_E_INVALID
    assert "scratch" in tf.lib().tf_last_error(g.ctx).decode()
    assert np.all(np.isnan(rows))                           # nothing was written
    ptr, oidx, vals = _batch(dims, [5000, 17], 8)           # a batch that fits still runs
    rc0, want, _ = _run(tf.lib().tf_foldin, g, ptr, oidx, vals, tf.TF_FOLDIN_FULL)
    rc1, got, _ = _run(tf.lib().tf_foldin_noalloc, g, ptr, oidx, vals, tf.TF_FOLDIN_FULL)
    assert rc0 == rc1 == tf.TF_OK and np.array_equal(got, want)
    g.close()
