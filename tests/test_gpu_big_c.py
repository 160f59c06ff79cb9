"""Splits wider than the narrow kernels take (17..128 columns in FP64,
33..128 in FP32 / BF16), through tf_sweep / tf_split on the GPU, against the
FP64 oracle.  C = K with T_in = 1 is the ALS row solve of eq. (ALS)
(Section 3.1), which the oracle is pinned to on the CPU.

Tolerances as for the narrow kernels: FP64 factors within 1e-10 of the
oracle (max-abs relative) and loss within 1e-9; FP32 loss and RMSE within
1e-4; BF16 loss within 1e-2 and RMSE within 5e-3."""
import numpy as np
import pytest

from gpu_util import note, pair, problem, rel_max

pytestmark = pytest.mark.gpu


def _compare(g, o, N, prec):
    gl, gr = g.loss()
    ol, orr = o.loss()
    if prec == "f64":
        for n in range(N):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
        assert abs(gl - ol) <= 1e-9 * ol
    elif prec == "f32":
        assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr, (gl, ol, gr, orr)
    else:
        assert abs(gr - orr) <= 5e-3 * orr and abs(gl - ol) <= 1e-2 * ol, (gl, ol, gr, orr)


@pytest.mark.parametrize("prec,K", [("f64", 20), ("f64", 40), ("f32", 100), ("bf16", 64),
                                    ("f64", 128)])
def test_als_sweep_c_equals_k(prec, K):
    """tf_sweep(C = K, T_in = 1): every row of every mode solved by eq. (ALS),
    on skewed rows (some cut into chunks) with repeated sweeps."""
    dims = [120, 90, 70]
    note(f"ALS C=K={K} {prec}")
    idx, x, A = problem(400 + K, dims, 9000, K, dist="zipf", dedupe="drop")
    g, o = pair(dims, idx, x, A, K, 0.5, prec, split_threshold=256, chunk_nnz=64)
    for _ in range(2):
        g.sweep(K, 1)
        o.sweep(K, 1)
    _compare(g, o, 3, prec)
    g.close()


@pytest.mark.parametrize("prec,K,C,T_in", [("f64", 50, 20, 2), ("f64", 40, 32, 1),
                                           ("f32", 100, 40, 2), ("f32", 72, 33, 1),
                                           ("bf16", 90, 45, 1)])
def test_wide_splits_mixed_with_narrow_ones(prec, K, C, T_in):
    """K not a multiple of C: wide splits followed by a narrower last split,
    which first takes the wide split's pending columns out of the residual;
    the loss in between reads the residual after a wide split."""
    dims = [80, 70, 60, 50]
    note(f"wide splits {prec} K={K} C={C} T_in={T_in}")
    idx, x, A = problem(420 + C, dims, 12000, K, dist="zipf", dedupe="drop", first_zero=False)
    A = [a * (1.0 / np.mean(A[1])) ** 0.5 for a in A]
    g, o = pair(dims, idx, x, A, K, 0.3, prec, split_threshold=512, chunk_nnz=128)
    g.sweep(C, T_in)
    o.sweep(C, T_in)
    _compare(g, o, 4, prec)
    cols = list(range(3, 3 + C))
    g.split(cols, 1)                 # a wide split right after the sweep's last one
    o.split(cols, 1)
    g.split([0, 1, 2], 1)            # and a narrow one after it
    o.split([0, 1, 2], 1)
    _compare(g, o, 4, prec)
    rg, ro = g.residual(), o.residual()
    # BF16 storage rounds every stored factor value to 8 significant bits
    # (relative 2^-9), which the residual x - recon inherits
    tol = {"f64": 1e-9, "f32": 1e-3, "bf16": 1e-2}[prec]
    assert np.max(np.abs(rg - ro)) <= tol * np.max(np.abs(x))
    g.close()


def test_wide_split_weighted_lambda_random_order_and_empty_rows_f64():
    """Weighted lambda |Omega_i| (Section 5.1.3), a random column permutation,
    and rows with no entries (set to zero), at C = 24 in FP64."""
    from paper_1410_5209_amd import tf
    import synth
    dims, K = [200, 60, 50], 48
    note("wide weighted random order f64")
    idx, x, A = problem(440, dims, 4000, K, first_zero=False)
    idx = idx[idx[:, 0] < 150]              # rows 150..199 of mode 0 have no entries
    x = x[: idx.shape[0]]
    g, o = pair(dims, idx, x, A, K, 0.05, "f64", reg_mode=1)
    order = synth.column_order(3, 0, K)
    g.set_col_order(order)
    g.sweep(24, 1)
    o.sweep(24, 1, order)
    _compare(g, o, 3, "f64")
    assert np.all(g.factor(0)[150:] == 0.0)
    g.close()


def test_c_above_the_limit_is_refused():
    from paper_1410_5209_amd import tf
    dims, K = [30, 20, 10], 130
    idx, x, A = problem(450, dims, 800, K)
    g, o = pair(dims, idx, x, A, K, 1.0, "f32")
    with pytest.raises(tf.TFError) as e:
        g.sweep(129, 1)
    assert e.value.status == tf.TF_E_UNSUPPORTED
    g.sweep(128, 1)                   # 128 columns, then the remaining 2
    o.sweep(128, 1)
    _compare(g, o, 3, "f32")
    g.close()
