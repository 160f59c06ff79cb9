"""CPU checks of the C-ABI library: it loads, exports every symbol include/tf.h
declares, its host-only row planner follows its rules, and host-side
argument validation rejects bad calls before any GPU work."""
import ctypes

import numpy as np
import pytest

from paper_1410_5209_amd import tf


def test_library_exports_every_declared_symbol():
    L = tf.lib()
    names = tf.declared_symbols()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


def test_options_struct_matches_header_defaults():
    o = tf.tf_default_options()
    assert o.size == ctypes.sizeof(tf.tf_options) == 104
    assert (o.precision, o.reg_mode, o.first_factor_zero, o.strategy, o.seed) == (1, 0, 1, 1, 2)
    assert (o.lane_nnz, o.split_threshold, o.chunk_nnz) == (2, 4096, 2048)
    assert o.resid_share == tf.TF_RESID_AUTO
    assert o.col_order == tf.TF_ORDER_FIXED and o.mem_budget == 0
    assert not o.dev_alloc and not o.dev_free and o.alloc_user is None
    assert o.graph == 0


def _rowptr(counts):
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def test_plan_plain_is_one_wavefront_per_nonempty_row():
    counts = [0, 5, 1, 0, 300, 7]
    s = tf.tf_plan_rows(_rowptr(counts), strategy=tf.TF_STRATEGY_PLAIN)
    assert s.tasks == 4 and s.empty_rows == 2 and s.split_rows == 0 and s.chunks == 0
    assert list(s.rows_by_lanes) == [0, 0, 0, 0, 0, 0, 4]


def test_plan_skew_buckets_and_chunks():
    # lane_nnz 8: G = smallest power of two >= ceil(cnt / 8), capped at 64;
    # rows longer than the split threshold are cut into ceil(cnt / chunk) chunks
    counts = [1, 8, 9, 16, 17, 100, 512, 513, 1000, 5000, 0, 12000]
    s = tf.tf_plan_rows(_rowptr(counts), lane_nnz=8, split_threshold=4096, chunk_nnz=2048)
    want_g = {1: 2, 2: 2, 4: 1, 16: 1, 64: 3}   # G -> rows: {1,8}->1, {9,16}->2, 17->4, 100->16,
    got = {1 << b: int(c) for b, c in enumerate(s.rows_by_lanes) if c}
    assert got == want_g
    assert s.split_rows == 2 and s.empty_rows == 1
    assert s.chunks == 3 + 6                      # 5000 -> 3 chunks, 12000 -> 6 chunks
    # tasks: 9 chunks + per bucket ceil(rows / (64 / G))
    assert s.tasks == 9 + 1 + 1 + 1 + 1 + 3


def test_plan_rejects_bad_offsets():
    with pytest.raises(tf.TFError):
        tf.tf_plan_rows(np.array([0, 3, 2], dtype=np.int64))


def test_init_rejects_bad_arguments_on_host():
    L = tf.lib()
    ctx = ctypes.c_void_p()
    dims = np.array([4, 4, 4], dtype=np.int64)
    fake = ctypes.c_void_p(16)    # never dereferenced: host checks fail first
    cases = [
        (1, dims, 10, 2, 1.0),        # N < 2
        (3, dims, 0, 2, 1.0),         # nnz < 1
        (3, dims, 10, 0, 1.0),        # K < 1
        (3, dims, 10, 2, 0.0),        # lambda must be > 0
        (3, dims, 10, 2, float("nan")),
        (3, np.array([4, 0, 4], dtype=np.int64), 10, 2, 1.0),
    ]
    for N, d, nnz, K, lam in cases:
        st = L.tf_init(ctypes.byref(ctx), N, d.ctypes.data_as(ctypes.c_void_p), nnz, fake, fake,
                       K, lam, None)
        assert st == tf.TF_E_INVALID, (N, nnz, K, lam)
        assert ctx.value is None
        assert len(tf.tf_last_error(None)) > 0
    bad_opts = [tf.tf_default_options(precision=7), tf.tf_default_options(strategy=4),
                tf.tf_default_options(col_order=2), tf.tf_default_options(resid_share=5),
                tf.tf_default_options(graph=2)]
    half = tf.tf_default_options()
    half.dev_alloc = tf.ALLOC_FN(lambda n, s, u: None)   # dev_free left NULL
    bad_opts.append(half)
    for o in bad_opts:
        st = L.tf_init(ctypes.byref(ctx), 3, dims.ctypes.data_as(ctypes.c_void_p), 10, fake, fake,
                       2, 1.0, ctypes.byref(o))
        assert st == tf.TF_E_INVALID and ctx.value is None
