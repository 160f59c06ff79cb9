"""The benchmark workloads' recipes at sizes the oracle follows, over their
full number of sweeps, and the longest-row cases of the planner, on the GPU
through the C ABI against the FP64 oracle.

* The 3-way workload (mode lengths 1M, 1e8 entries, K = 100, C = 10,
  T_in = 2, 10 sweeps) as a replica with mode lengths 3000 and 3e5 entries
  (mean row length 100, as at full size) from the same generator: every one
  of the 10 sweeps (10 splits each) must keep the loss and training RMSE
  within 1e-4 relative of the oracle in FP32, and within the BF16 bounds
  (loss 1e-2, RMSE 5e-3) with BF16 factors.
* A row cut into more chunks than the planner allows per row (1024), whose
  chunks are lengthened instead: 3e5 entries in one row with 64-entry
  chunks, at C = 10 (register kernel), C = 32 (matrix-core kernel) and, in
  FP64, C = 32 (workgroup-per-row kernel)."""
import numpy as np
import pytest

import synth
from gpu_util import note, pair, rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["sals-3way-1m-fp32", "sals-3way-1m-bf16"])
def test_benchmark_recipe_replica_ten_sweeps(name):
    w = synth.WORKLOADS[name].replica(3000, 300_000)
    note(f"replica {w.name}: K={w.K} C={w.C} T_in={w.T_in} {w.sweeps} sweeps {w.prec}")
    data = synth.make_tensor(w)
    idx, x = data[0], data[1]
    A = synth.factors(synth.SEED_INIT, w.dims, w.K, first_zero=True)
    g, o = pair(w.dims, idx, x, A, w.K, w.lam, w.prec)
    g.autotune(w.T_in, [w.C], tune_tiles=True)
    tl, tr = (1e-4, 1e-4) if w.prec == "f32" else (1e-2, 5e-3)
    worst_l = worst_r = 0.0
    for s in range(w.sweeps):
        g.sweep(w.C, w.T_in)
        o.sweep(w.C, w.T_in)
        gl, gr = g.loss()
        ol, orr = o.loss()
        worst_l = max(worst_l, abs(gl - ol) / ol)
        worst_r = max(worst_r, abs(gr - orr) / orr)
        assert abs(gl - ol) <= tl * ol and abs(gr - orr) <= tr * orr, (s, gl, ol, gr, orr)
    note(f"replica {w.name}: worst loss {worst_l:.3g} RMSE {worst_r:.3g} over {w.sweeps} sweeps")
    g.close()


def _one_heavy_row(seed, dims, heavy, rest):
    other = [synth.uniform_ints(seed, 70 + t, heavy, dims[t + 1]) for t in range(2)]
    h = np.stack([np.zeros(heavy, np.int32), other[0], other[1]], axis=1).astype(np.int32)
    r = synth.tuples(seed, dims, rest)
    idx = np.concatenate([h, r[r[:, 0] != 0]]).astype(np.int32)
    x = synth.values(seed, dims, idx, 3, 0, 0.1)
    return idx, x


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,C", [("f32", 10), ("f32", 32), ("f64", 10), ("f64", 32)])
def test_row_beyond_the_chunk_cap(prec, C):
    from paper_1410_5209_amd import tf
    dims, K = [40, 3000, 3000], 40
    note(f"heavy row {prec} C={C}")
    idx, x = _one_heavy_row(77, dims, 300_000, 20_000)
    rp = np.concatenate([[0], np.cumsum(np.bincount(idx[:, 0], minlength=dims[0]))])
    plan = tf.tf_plan_rows(rp.astype(np.int64), strategy=tf.TF_STRATEGY_SKEW, lane_nnz=2,
                           split_threshold=128, chunk_nnz=64)
    assert plan.chunks >= 1024 and plan.split_rows >= 1
    A = synth.factors(78, dims, K, first_zero=True)
    g, o = pair(dims, idx, x, A, K, 0.5, prec, split_threshold=128, chunk_nnz=64)
    cols = list(range(5, 5 + C))
    for T_in in (2, 1):
        g.split(cols, T_in)
        o.split(cols, T_in)
    gl, gr = g.loss()
    ol, orr = o.loss()
    if prec == "f64":
        for n in range(3):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
        assert abs(gl - ol) <= 1e-9 * ol
    else:
        assert rel_max(g.factor(0)[0], o.get_factor(0)[0]) < 1e-3
        assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr, (gl, ol, gr, orr)
    g.close()
