"""GPU path vs the FP64 oracle on the same seeded inputs, through the C ABI.

Tolerances: CSR and indexing bit-exact; FP64 mode factors within 1e-10
(max-abs, relative to the largest entry) and loss within 1e-9 relative;
FP32 mode RMSE and loss within 1e-4 relative (FP32 accumulation over a few
hundred terms per row and FP32 residual storage give ~1e-6 per step)."""
import numpy as np
import pytest

import synth
from gpu_util import note, pair, problem, recon, rel_max

pytestmark = pytest.mark.gpu

PLAIN, SKEW = 0, 1


# ------------------------------------------------------------------ CSR

@pytest.mark.parametrize("case", ["uniform", "multiset", "zipf", "empty_rows", "one_row"])
def test_csr_bit_exact(case):
    from oracle import oracle as orc
    from paper_1410_5209_amd.model import SparseCP
    if case == "uniform":
        dims, idx = [300, 200, 100], synth.tuples(1, [300, 200, 100], 20000)
    elif case == "multiset":
        dims, idx = [7, 5, 3], synth.tuples(2, [7, 5, 3], 5000, dedupe="none")
    elif case == "zipf":
        dims, idx = [5000, 4000, 3000, 2000], synth.tuples(3, [5000, 4000, 3000, 2000], 60000,
                                                           dist="zipf", dedupe="drop")
    elif case == "empty_rows":
        dims = [100000, 50, 70000]
        idx = synth.tuples(4, [1000, 50, 700], 3000)
        idx[:, 0] *= 97
        idx[:, 2] *= 99
    else:
        dims = [1 << 20, 3]
        idx = np.stack([np.full(9000, 777777, dtype=np.int32),
                        synth.uniform_ints(5, 1, 9000, 3)], axis=1)
    note(f"csr {case} dims={dims} nnz={idx.shape[0]}")
    x = np.zeros(idx.shape[0])
    g = SparseCP(dims, idx, x, 2, 1.0, precision="f64")
    o = orc.Oracle(dims, idx, x, 2, 1.0)
    for n in range(len(dims)):
        rp, pm = g.csr(n)
        orp, opm = o.get_csr(n)
        assert np.array_equal(rp, orp) and np.array_equal(pm, opm)
    g.close()


# --------------------------------------------------------- FP64 split parity

SPLIT_CASES = [
    # N, dims, nnz, K, cols, T_in, reg, strategy
    (3, [60, 50, 40], 3000, 6, [0], 1, 0, SKEW),                 # CDTF
    (3, [60, 50, 40], 3000, 6, [2, 5, 1], 2, 0, SKEW),
    (3, [60, 50, 40], 3000, 10, list(range(10)), 1, 0, SKEW),    # C = K: ALS
    (2, [90, 70], 2500, 5, [4, 3, 2, 1], 1, 1, SKEW),            # weighted lambda
    (4, [30, 25, 20, 15], 4000, 8, [7, 0, 3, 5, 1, 6], 2, 0, PLAIN),
    (5, [20, 18, 16, 14, 12], 5000, 4, [1, 2], 1, 1, SKEW),
    (8, [6, 5, 6, 5, 6, 5, 6, 5], 3000, 3, [0, 2], 1, 0, SKEW),
    (3, [400, 300, 5], 20000, 16, list(range(3, 16)), 1, 0, SKEW),  # long rows of mode 2
]


@pytest.mark.parametrize("N,dims,nnz,K,cols,T_in,reg,strategy", SPLIT_CASES)
def test_split_parity_f64(N, dims, nnz, K, cols, T_in, reg, strategy):
    note(f"split f64 N={N} dims={dims} K={K} C={len(cols)} T_in={T_in} reg={reg} strat={strategy}")
    idx, x, A = problem(100 + N, dims, nnz, K)
    g, o = pair(dims, idx, x, A, K, 0.2, "f64", reg, strategy=strategy, split_threshold=512,
                chunk_nnz=128)
    for _ in range(2):
        g.split(cols, T_in)
        o.split(cols, T_in)
        for n in range(N):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
        assert np.max(np.abs(g.residual() - o.residual())) < 1e-10 * np.max(np.abs(x))
        gl, gr = g.loss()
        ol, orr = o.loss()
        assert abs(gl - ol) <= 1e-9 * ol and abs(gr - orr) <= 1e-9 * orr
    g.close()


def test_changing_split_width_f64():
    """Splits narrower than the previous one run at the previous width with
    zero-padded columns, keeping the residual update fused."""
    dims, K = [50, 40, 30], 12
    note("split width change f64")
    idx, x, A = problem(7, dims, 4000, K)
    g, o = pair(dims, idx, x, A, K, 0.3, "f64")
    for cols in ([0, 1, 2, 3, 4, 5, 6, 7, 8, 9], [10], [11, 3], list(range(12)), [5]):
        g.split(cols, 1)
        o.split(cols, 1)
        for n in range(3):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10
    gl, _ = g.loss()
    ol, _ = o.loss()
    assert abs(gl - ol) <= 1e-9 * ol
    g.close()


@pytest.mark.parametrize("share", ["own", "shared", "auto"])
def test_residual_placement_f64(share):
    """Modes 2..N keep their own R-hat or read mode 1's through a permutation;
    widths alternate so that the automatic choice switches back and forth
    (a mode returning to its own copy takes mode 1's R-hat first)."""
    from paper_1410_5209_amd import tf
    mode = {"own": tf.TF_RESID_OWN, "shared": tf.TF_RESID_SHARED, "auto": tf.TF_RESID_AUTO}[share]
    dims, K = [40, 35, 30, 25], 24
    note(f"residual placement f64 {share}")
    idx, x, A = problem(17, dims, 5000, K)
    g, o = pair(dims, idx, x, A, K, 0.2, "f64", resid_share=mode)
    plan = [(list(range(16)), 1), ([16, 17, 18], 1), (list(range(8, 24)), 2), ([0, 5, 9, 13, 2], 1),
            (list(range(12)), 1), ([23], 2)]
    for cols, t_in in plan:
        g.split(cols, t_in)
        o.split(cols, t_in)
        for n in range(4):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, (cols, n)
    assert rel_max(g.residual(), o.residual()) < 1e-10
    gl, _ = g.loss()
    ol, _ = o.loss()
    assert abs(gl - ol) <= 1e-9 * ol
    g.close()


def test_sweeps_with_random_column_orders_f64():
    dims, K, C = [80, 70, 60], 9, 4
    note("sweeps random order f64")
    idx, x, A = problem(8, dims, 6000, K)
    g, o = pair(dims, idx, x, A, K, 0.1, "f64")
    for s in range(3):
        order = synth.column_order(synth.SEED_ORDER, s, K)
        g.set_col_order(order)
        g.sweep(C, 2)
        o.sweep(C, 2, order)
        gl, _ = g.loss()
        ol, _ = o.loss()
        assert abs(gl - ol) <= 1e-9 * ol
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-9
    g.close()


def test_cdtf_1k_workload_ten_sweeps_f64():
    """The CDTF workload: 3-way 1000^3, 1e5 distinct uniform entries, rank-10
    truth + N(0, 0.1^2), K = 10, lambda = 0.1, C = 1, 10 sweeps, FP64."""
    w = synth.WORKLOADS["cdtf-3way-1k-fp64"]
    note("cdtf 1k workload f64, 10 sweeps")
    idx, x = synth.make_tensor(w)
    dims = [w.I] * w.N
    A = synth.factors(synth.SEED_INIT, dims, w.K, first_zero=True)
    g, o = pair(dims, idx, x, A, w.K, w.lam, "f64")
    prev = None
    for s in range(w.sweeps):
        g.sweep(w.C, w.T_in)
        o.sweep(w.C, w.T_in)
        gl, gr = g.loss()
        ol, orr = o.loss()
        assert abs(gl - ol) <= 1e-9 * ol, (s, gl, ol)
        assert prev is None or gl <= prev * (1 + 1e-12)
        prev = gl
    assert rel_max(g.residual(), o.residual()) < 1e-9
    g.close()


def test_loss_never_increases_each_split_f64():
    dims, K = [120, 100, 80], 8
    note("monotone loss f64")
    idx, x, A = problem(9, dims, 9000, K)
    g, _ = pair(dims, idx, x, A, K, 0.05, "f64")
    prev = g.loss()[0]
    for cols in ([0, 1, 2], [3, 4, 5], [6, 7], [1], [0, 2, 4, 6]):
        g.split(cols, 2)
        cur = g.loss()[0]
        assert cur <= prev * (1 + 1e-12)
        prev = cur
    F = g.factors()
    assert np.max(np.abs(g.residual() - (x - recon(dims, idx, F)))) < 1e-10 * np.max(np.abs(x))
    g.close()


# ------------------------------------------------------------ FP32 / BF16

def _reduced_3way(scale_I, nnz, K):
    w = synth.WORKLOADS["sals-3way-1m-fp32"].replica(scale_I, nnz, K=K)
    idx, x = synth.make_tensor(w)
    dims = [w.I] * 3
    A = synth.factors(synth.SEED_INIT, dims, w.K, first_zero=True)
    return w, dims, idx, x, A


@pytest.mark.parametrize("strategy", [PLAIN, SKEW])
def test_f32_reduced_3way_parity(strategy):
    w, dims, idx, x, A = _reduced_3way(3000, 300_000, 20)
    note(f"f32 reduced 3-way strategy={strategy}")
    g, o = pair(dims, idx, x, A, w.K, w.lam, "f32", strategy=strategy)
    for s in range(3):
        g.sweep(w.C, w.T_in)
        o.sweep(w.C, w.T_in)
        gl, gr = g.loss()
        ol, orr = o.loss()
        assert abs(gr - orr) <= 1e-4 * orr, (s, gr, orr)
        assert abs(gl - ol) <= 1e-4 * ol, (s, gl, ol)
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3
    g.close()


def test_bf16_reduced_3way_stays_close():
    """BF16 factor storage rounds every stored value to 8 significant bits
    (relative step 2^-8); the loss stays within 1% of the FP64 oracle and the
    RMSE within 0.5% over three sweeps."""
    w, dims, idx, x, A = _reduced_3way(3000, 300_000, 20)
    note("bf16 reduced 3-way")
    g, o = pair(dims, idx, x, A, w.K, w.lam, "bf16")
    for s in range(3):
        g.sweep(w.C, w.T_in)
        o.sweep(w.C, w.T_in)
    gl, gr = g.loss()
    ol, orr = o.loss()
    assert abs(gr - orr) <= 5e-3 * orr
    assert abs(gl - ol) <= 1e-2 * ol
    g.close()


# ---------------------------------------------------------------- skew

def test_zipf_skewed_split_rows_f64_and_determinism():
    dims, K = [3000, 2500, 2000], 6
    note("zipf skew f64 with split rows")
    idx, x, A = problem(11, dims, 80000, K, dist="zipf", dedupe="drop")
    g, o = pair(dims, idx, x, A, K, 0.5, "f64", split_threshold=256, chunk_nnz=64)
    g.split([0, 1, 2, 3, 4, 5], 1)
    o.split([0, 1, 2, 3, 4, 5], 1)
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10
    F1 = g.factors()
    g.set_factors(A)
    g.split([0, 1, 2, 3, 4, 5], 1)
    for n in range(3):
        assert np.array_equal(g.factor(n), F1[n])      # bitwise reproducible
    g.close()


# --------------------------------------------------------------- predict

def test_predict_and_invalid_query():
    from paper_1410_5209_amd import tf
    dims, K = [40, 30, 20], 5
    note("predict")
    idx, x, A = problem(12, dims, 2000, K, first_zero=False)
    g, o = pair(dims, idx, x, A, K, 0.2, "f64")
    q = synth.tuples(13, dims, 500, dedupe="none")
    assert rel_max(g.predict(q), o.predict(q)) < 1e-14
    bad = q.copy()
    bad[7, 2] = dims[2]
    with pytest.raises(tf.TFError):
        g.predict(bad)
    g.close()


def test_init_rejects_out_of_range_index_and_nan():
    from paper_1410_5209_amd import tf
    from paper_1410_5209_amd.model import SparseCP
    note("init validation")
    idx = synth.tuples(14, [10, 10, 10], 100)
    x = np.ones(100)
    bad = idx.copy()
    bad[42, 1] = 10
    with pytest.raises(tf.TFError, match="entry 42"):
        SparseCP([10, 10, 10], bad, x, 2, 1.0)
    xb = x.copy()
    xb[17] = np.inf
    with pytest.raises(tf.TFError, match="entry 17"):
        SparseCP([10, 10, 10], idx, xb, 2, 1.0)


def test_library_init_draws_splitmix_factors():
    from oracle import oracle as orc
    from paper_1410_5209_amd.model import SparseCP
    note("library factor init")
    dims, K = [30, 20, 10], 7
    idx = synth.tuples(15, dims, 500)
    x = synth.values(15, dims, idx, 3, 0, 0.1)
    o = orc.Oracle(dims, idx, x, K, 1.0)
    for fz in (True, False):
        g = SparseCP(dims, idx, x, K, 1.0, precision="f64", first_factor_zero=fz, seed=99)
        o.init_factors(99, fz)
        for n in range(3):
            assert np.array_equal(g.factor(n), o.get_factor(n))
        o.resync()
        assert rel_max(g.residual(), o.residual()) < 1e-14 or np.array_equal(g.residual(), x)
        g.close()


# ------------------------------------------------------ 32-column splits

@pytest.mark.parametrize("N,dims,nnz,dist", [
    (3, [300, 250, 200], 30000, "uniform"),
    (5, [60, 50, 40, 30, 20], 30000, "uniform"),
    (5, [400, 300, 300, 200, 200], 40000, "zipf"),
])
def test_wide_split_parity_f32(N, dims, nnz, dist):
    """C = 32 (half a wavefront per entry, Gram on the matrix cores), then a
    split of 8 columns whose pending 32 columns exceed that kernel's width."""
    K = 40
    note(f"wide f32 N={N} dims={dims} dist={dist}")
    idx, x, A = problem(200 + N, dims, nnz, K, dist=dist,
                        dedupe="drop" if dist == "zipf" else "distinct")
    g, o = pair(dims, idx, x, A, K, 0.5, "f32", split_threshold=512, chunk_nnz=200)
    for cols in (list(range(32)), list(range(32, 40)), list(range(4, 36))):
        g.split(cols, 1)
        o.split(cols, 1)
        gl, gr = g.loss()
        ol, orr = o.loss()
        assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr, (cols[0], gl, ol)
        for n in range(N):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3, n
    g.close()


def test_wide_sweep_bf16_and_t_in_2():
    dims, K = [200, 150, 100], 64
    note("wide bf16 sweep")
    idx, x, A = problem(210, dims, 20000, K)
    g, o = pair(dims, idx, x, A, K, 0.5, "bf16")
    g.sweep(32, 2)
    o.sweep(32, 2)
    gl, gr = g.loss()
    ol, orr = o.loss()
    assert abs(gr - orr) <= 5e-3 * orr and abs(gl - ol) <= 1e-2 * ol
    g.close()


@pytest.mark.parametrize("C,T_in", [(1, 1), (5, 2), (8, 1)])
def test_short_mode_shape_f64(C, T_in):
    """The aspect of the paper's Netflix_3 tensor (one long mode, one very
    short one): the 7 rows of mode 3 hold ~8.6k entries each and are cut into
    chunks whose partial Grams are summed in a fixed order."""
    dims, K = [3000, 200, 7], 8
    note(f"short-mode shape f64 C={C} T_in={T_in}")
    idx, x, A = problem(41, dims, 60000, K)
    g, o = pair(dims, idx, x, A, K, 0.02, "f64", split_threshold=1024, chunk_nnz=512)
    g.sweep(C, T_in)
    o.sweep(C, T_in)
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
    gl, _ = g.loss()
    ol, _ = o.loss()
    assert abs(gl - ol) <= 1e-9 * ol
    g.close()


def test_four_mode_short_tail_shape_wide_f32():
    """The aspect of the paper's Yahoo-music_4 tensor (two long modes, two
    short ones) at K = 40, C = 20: the split runs at 32 columns with zero
    padding on the wide kernel, with chunked long rows in modes 3 and 4."""
    dims, K = [2000, 1500, 20, 6], 40
    note("four-mode short tail wide f32")
    idx, x, A = problem(42, dims, 80000, K)
    g, o = pair(dims, idx, x, A, K, 1.0, "f32", split_threshold=2048, chunk_nnz=1024)
    g.sweep(20, 1)
    o.sweep(20, 1)
    gl, gr = g.loss()
    ol, orr = o.loss()
    assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr, (gl, ol)
    for n in range(4):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3, n
    g.close()


def test_autotune_leaves_model_unchanged_and_sweeps_with_chosen_width():
    dims, K = [400, 300, 200], 40
    note("autotune")
    idx, x, A = problem(220, dims, 40000, K, dist="zipf", dedupe="drop")
    g, o = pair(dims, idx, x, A, K, 0.5, "f32", split_threshold=512, chunk_nnz=128)
    g.split(list(range(8)), 1)
    o.split(list(range(8)), 1)
    F0, r0 = g.factors(), g.residual()
    res = g.autotune(1, [4, 8, 16, 32], tune_tiles=True)
    assert res.best_C in (4, 8, 16, 32) and res.ncand == 4
    assert all(res.est_sweep_ms[q] > 0 for q in range(4))
    assert all(res.lane_nnz[n] in (1, 2, 4, 8) for n in range(3))
    assert all(res.persistent[n] in (0, 1) for n in range(3))
    for n in range(3):
        assert np.array_equal(g.factor(n), F0[n])
    assert np.array_equal(g.residual(), r0)
    g.sweep(0, 1)
    order = np.arange(K)
    o.sweep(res.best_C, 1, order)
    gl, gr = g.loss()
    ol, orr = o.loss()
    assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr
    g.close()


@pytest.mark.parametrize("case", ["one_entry", "rank_one", "matrix_als"])
def test_degenerate_sizes_f64(case):
    """A tensor with a single entry (all other rows of every mode empty), rank
    K = 1 (every split is the C = 1 update), and a 2-way matrix at C = K."""
    if case == "one_entry":
        dims, nnz, K, C, T_in = [5, 4, 3], 1, 3, 3, 1
    elif case == "rank_one":
        dims, nnz, K, C, T_in = [30, 20, 10], 500, 1, 1, 2
    else:
        dims, nnz, K, C, T_in = [70, 50], 2000, 6, 6, 1
    note(f"degenerate {case} dims={dims} nnz={nnz} K={K}")
    idx, x, A = problem(300, dims, nnz, K)
    g, o = pair(dims, idx, x, A, K, 0.3, "f64")
    for _ in range(2):
        g.sweep(C, T_in)
        o.sweep(C, T_in)
        for n in range(len(dims)):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
    gl, _ = g.loss()
    ol, _ = o.loss()
    assert abs(gl - ol) <= 1e-9 * ol
    g.close()


def test_factor_block_reads_chosen_rows_and_columns():
    from paper_1410_5209_amd import tf
    dims, K = [50, 40, 30], 12
    note("factor block")
    idx, x, A = problem(301, dims, 3000, K)
    for prec in ("f64", "f32", "bf16"):
        g, _ = pair(dims, idx, x, A, K, 0.3, prec)
        g.split([0, 1, 2, 3], 1)
        F = g.factor(1)
        rows, cols = np.array([39, 0, 7, 7]), np.array([11, 2, 2])
        assert np.array_equal(g.factor_block(1, rows, cols), F[rows][:, cols])
        assert np.array_equal(g.factor_block(1, rows, None), F[rows])
        assert np.array_equal(g.factor_block(1, None, cols), F[:, cols])
        assert np.array_equal(g.factor_block(1), F)
        for bad in (dict(rows=[40]), dict(cols=[12]), dict(rows=[-1]), dict(cols=[])):
            with pytest.raises(tf.TFError) as e:
                g.factor_block(1, bad.get("rows"), bad.get("cols"))
            assert e.value.status == tf.TF_E_INVALID
        g.close()


def test_non_positive_pivot_is_reported_and_recovered_f64():
    """A factor row of 1e200 overflows the Gram matrices of the mode-1 rows it
    meets (B = Inf, so the Cholesky pivots become NaN): the sweep reports
    TF_E_NUMERIC naming mode 0 and the smallest such row, as the oracle does;
    those rows keep their values and every other mode-1 row is updated as by
    the oracle; tf_set_factor + tf_resync then restore a state that sweeps
    like a fresh oracle."""
    import re
    from oracle import oracle as orc
    from paper_1410_5209_amd import tf
    dims, K = [40, 30, 20], 4
    note("non-positive pivot f64")
    idx, x, A = problem(320, dims, 3000, K, first_zero=False)
    bad = [a.copy() for a in A]
    bad[1][3, :] = 1e200
    g, o = pair(dims, idx, x, bad, K, 0.3, "f64")
    with pytest.raises(tf.TFError) as e:
        g.sweep(K, 1)
    assert e.value.status == tf.TF_E_NUMERIC
    m = re.search(r"mode (\d+) row (\d+)", str(e.value))
    with pytest.raises(orc.OracleError) as oe:
        o.sweep(K, 1)
    obad = int(re.search(r"bad_row=(\d+)", str(oe.value)).group(1))
    assert m and int(m.group(1)) == 0 and int(m.group(2)) == obad
    touched = np.unique(idx[idx[:, 1] == 3, 0])
    assert int(m.group(2)) == touched.min()
    G0, O0 = g.factor(0), o.get_factor(0)
    assert np.array_equal(G0[touched], bad[0][touched])
    keep = np.setdiff1d(np.arange(dims[0]), touched)
    assert rel_max(G0[keep], O0[keep]) < 1e-10
    g.set_factors(A)
    o2 = orc.Oracle(dims, idx, x, K, 0.3)
    for n, An in enumerate(A):
        o2.set_factor(n, An)
    o2.resync()
    g.sweep(K, 1)
    o2.sweep(K, 1)
    for n in range(3):
        assert rel_max(g.factor(n), o2.get_factor(n)) < 1e-10, n
    g.close()


@pytest.mark.parametrize("share", ["own", "shared"])
def test_pivot_failure_in_a_later_split_stops_the_sweep_as_the_oracle_f64(share):
    """K = 8, C = 3: blocks (0,1,2), (3,4,5), (6,7).  Mode 1's row 3 holds 1e200
    in columns 3..5 and A^(1) = 0, so the first block runs normally and the
    second block's mode-0 rows that meet that row get an infinite Gram
    matrix.  The oracle stops its sweep after that mode pass (those rows keep
    their values, the pass's other rows are updated, nothing after it
    changes); the library must leave the same factors and residual and name
    the same mode and smallest row."""
    import re
    from oracle import oracle as orc
    from paper_1410_5209_amd import tf
    dims, K = [40, 30, 20], 8
    note(f"pivot failure in split 2 ({share})")
    mode = {"own": tf.TF_RESID_OWN, "shared": tf.TF_RESID_SHARED}[share]
    idx, x, A = problem(322, dims, 3000, K, first_zero=True)
    A[1][3, 3:6] = 1e200
    g, o = pair(dims, idx, x, A, K, 0.3, "f64", resid_share=mode)
    with pytest.raises(tf.TFError) as e:
        g.sweep(3, 2)
    assert e.value.status == tf.TF_E_NUMERIC
    m = re.search(r"mode (\d+) row (\d+)", str(e.value))
    with pytest.raises(orc.OracleError) as oe:
        o.sweep(3, 2)
    obad = int(re.search(r"bad_row=(\d+)", str(oe.value)).group(1))
    touched = np.unique(idx[idx[:, 1] == 3, 0])
    assert m and int(m.group(1)) == 0 and int(m.group(2)) == obad == touched.min()
    for n in range(3):
        G, O = g.factor(n), o.get_factor(n)
        keep = np.ones(dims[n], bool)
        if n == 1:
            keep[3] = False
            assert np.array_equal(G[3, 3:], O[3, 3:])          # untouched huge values
            assert rel_max(G[3, :3], O[3, :3]) < 1e-10
        assert rel_max(G[keep], O[keep]) < 1e-10, n
        assert np.array_equal(G[:, 6:], A[n][:, 6:])           # third block never updated
    G0 = g.factor(0)
    assert np.array_equal(G0[touched][:, 3:6], A[0][touched][:, 3:6])
    rg, ro = g.residual(), o.residual()
    assert np.max(np.abs(rg - ro)) < 1e-9 * np.max(np.abs(x))
    g.close()


@pytest.mark.parametrize("precision,share", [("f32", "own"), ("f32", "shared"), ("bf16", "own")])
def test_wide_split_with_each_residual_placement(precision, share):
    """C = 32 with every mode keeping its own R-hat (each mode's first pass reads
    the split-start segments of the modes already updated) or all reading mode
    1's copy, over two inner iterations and a following narrower split."""
    from paper_1410_5209_amd import tf
    mode = {"own": tf.TF_RESID_OWN, "shared": tf.TF_RESID_SHARED}[share]
    dims, K = [300, 250, 200, 150], 40
    note(f"wide {precision} placement {share}")
    idx, x, A = problem(340, dims, 30000, K, dist="zipf", dedupe="drop")
    g, o = pair(dims, idx, x, A, K, 0.5, precision, resid_share=mode, split_threshold=512,
                chunk_nnz=128)
    for cols, T_in in ((list(range(32)), 2), (list(range(32, 40)), 1), (list(range(5, 37)), 1)):
        g.split(cols, T_in)
        o.split(cols, T_in)
    gl, gr = g.loss()
    ol, orr = o.loss()
    if precision == "f32":
        assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr, (gl, ol)
        for n in range(4):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3, n
    else:
        assert abs(gr - orr) <= 5e-3 * orr and abs(gl - ol) <= 1e-2 * ol, (gl, ol)
    g.close()


WIDTH_CASES = [
    # precision, N, C, dist
    ("f32", 3, 1, "uniform"), ("f32", 3, 5, "zipf"), ("f32", 6, 12, "uniform"),
    ("f32", 7, 32, "zipf"), ("bf16", 4, 4, "zipf"), ("bf16", 3, 16, "uniform"),
    ("f64", 6, 3, "zipf"), ("f64", 3, 12, "uniform"),
]


@pytest.mark.parametrize("precision,N,C,dist", WIDTH_CASES)
def test_kernel_widths_and_mode_counts(precision, N, C, dist):
    """Compute widths and numbers of other modes not covered above (each an
    instantiation of its own), on uniform and skewed tensors with chunked
    rows, one split of two inner iterations against the oracle."""
    dims = [60, 50, 45, 40, 35, 30, 25][:N]
    K = max(C + 3, 8)
    note(f"widths {precision} N={N} C={C} {dist}")
    idx, x, A = problem(350 + N + C, dims, 12000, K, dist=dist,
                        dedupe="drop" if dist == "zipf" else "distinct", first_zero=False)
    # with five or more other modes, products of U(0,1)/sqrt(K) entries are so
    # small that lambda would drive every row towards zero within one split
    # (values below FP32's range); scale the factors to mean 1 and ease lambda
    scale = (1.0 / np.mean(A[1])) ** 0.5 if N > 4 else 1.0
    A = [a * scale for a in A]
    lam = 0.4 if N <= 4 else 0.02
    g, o = pair(dims, idx, x, A, K, lam, precision, split_threshold=256, chunk_nnz=64)
    cols = list(range(K - C, K))
    g.split(cols, 2)
    o.split(cols, 2)
    gl, gr = g.loss()
    ol, orr = o.loss()
    if precision == "f64":
        for n in range(N):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-10, n
        assert abs(gl - ol) <= 1e-9 * ol
    elif precision == "f32":
        for n in range(N):
            assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3, n
        assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr
    else:
        assert abs(gr - orr) <= 5e-3 * orr and abs(gl - ol) <= 1e-2 * ol, (gl, ol)
    g.close()


def test_wide_split_weighted_lambda_f32():
    """The 32-column kernels and solve with the weighted regulariser
    lambda |Omega_i| (Section 5.1.3), on skewed rows with chunks."""
    dims, K = [400, 300, 200], 40
    note("wide f32 weighted lambda")
    idx, x, A = problem(360, dims, 30000, K, dist="zipf", dedupe="drop", first_zero=False)
    g, o = pair(dims, idx, x, A, K, 0.05, "f32", reg_mode=1, split_threshold=512, chunk_nnz=128)
    for cols in (list(range(32)), list(range(8, 40))):
        g.split(cols, 1)
        o.split(cols, 1)
    for n in range(3):
        assert rel_max(g.factor(n), o.get_factor(n)) < 1e-3, n
    gl, gr = g.loss()
    ol, orr = o.loss()
    assert abs(gl - ol) <= 1e-4 * ol and abs(gr - orr) <= 1e-4 * orr
    g.close()
