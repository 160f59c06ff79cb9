"""Checks at the full sizes of the benchmark workloads, in the configuration the
benchmark times (tuned C and row tiles, a whole sweep), on properties that hold
at any size, since the oracle cannot follow 1e8-entry tensors.

* CSR (Table 1's row sets): the mode-n permutation is the stable sort of the
  entry ids by row: rows nondecreasing along it, ids strictly increasing inside
  a row, row counts and row pointers equal to the counts of the input indices.
  Together these fix the permutation uniquely; checked bit-exact.
* Split optimality (eq. (SALS)): after a split's last update of mode n each row
  of mode n minimises the split's regularised least squares with the other
  factors fixed, so its gradient vanishes:
  sum_{j in Omega_i} r_j p_j = lambda a_i, with r the maintained residual and
  p_j the elementwise product of the other modes' split columns at entry j.
  Checked on sampled rows of the last mode, long rows (several workgroups per
  row, and on the 5-way tensor rows of up to 2e6 entries and one whose chunks
  are lengthened to keep 1024 per row) among them, to 1e-4 of the summed
  magnitudes of the terms: FP32 storage
  and accumulation leave ~1e-6, a wrong, missing or misplaced term leaves O(1),
  a dropped lambda term O(1e-2) on the short rows.
* Residual (R, Section 3.1): r_j = x_j - sum_k prod_n a^(n)_{i_n k} on sampled
  entries, factors read back from the GPU and the sum taken in FP64 on the host,
  to 1e-4 of |x_j| + sum_k prod_n |a^(n)_{i_n k}| (FP32 storage, K/C
  incremental updates per sweep).  Predictions (tf_predict) on the same entries
  to the same bound.
* Loss (eq. (TF), 3-way): tf_loss equals sum r^2 + lambda sum_n ||A^(n)||_F^2
  recomputed on the host from the read-back residual and factors, to 1e-10.
* Fold-in (3-way): 200 requests of new mode-1 rows (Zipf sizes up to 5000
  entries) solved against the resident 1M-row factors, full rank and CDTF x 3,
  each against the oracle holding the same factors, to 1e-4 (FP32 Gram).
* BF16 factors (3-way, the workload with the held-out split): the same split
  optimality to 1e-2 (the stored rows are the FP64 solutions rounded to BF16:
  ~2^-9 of the scale) and the residual to 1e-4.
"""
import numpy as np
import pytest

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _check_csr(m, idx, n, I):
    rp, pm = m.csr(n)
    col = np.ascontiguousarray(idx[:, n])
    counts = np.bincount(col, minlength=I)
    assert rp.shape[0] == I + 1 and rp[0] == 0
    assert np.array_equal(rp[1:], np.cumsum(counts)), f"mode {n}: row pointers"
    assert pm.min() >= 0 and pm.max() < idx.shape[0], f"mode {n}: ids out of range"
    rows = col[pm]
    del col
    assert np.all(rows[1:] >= rows[:-1]), f"mode {n}: rows not sorted along the permutation"
    assert np.array_equal(np.bincount(rows, minlength=I), counts), f"mode {n}: row counts"
    same = rows[1:] == rows[:-1]
    del rows
    assert np.all(np.diff(pm)[same] > 0), f"mode {n}: ids not increasing inside a row"
    return rp, pm


def _rows_to_check(rp, rng, n_random, n_long, long_range, cap_len):
    lens = np.diff(rp)
    nonempty = np.flatnonzero(lens > 0)
    pick = [rng.choice(nonempty, size=min(n_random, nonempty.size), replace=False)]
    lo, hi = long_range
    longs = np.flatnonzero((lens >= max(lo, 1)) & (lens <= hi))
    if n_long and longs.size:
        pick.append(rng.choice(longs, size=min(n_long, longs.size), replace=False))
    capped = np.flatnonzero(lens <= cap_len)
    if capped.size:
        pick.append(capped[np.argsort(lens[capped], kind="stable")[-3:]])  # the longest ones
    return np.unique(np.concatenate(pick)).astype(np.int64)


def _gather_products(m, idx, J, skip, cols):
    """p_j over the modes other than `skip`, for entries J, columns cols."""
    P = np.ones((J.shape[0], len(cols) if cols is not None else m.K))
    for t in range(m.N):
        if t == skip:
            continue
        u, inv = np.unique(idx[J, t], return_inverse=True)
        P *= m.factor_block(t, u, cols)[inv]
    return P


def _pieces(rp, rows, batch):
    """Windows of at most `batch` entries over the listed rows (a long row is
    cut across windows): lists of (row slot, first position, end position)."""
    win, tot = [], 0
    for k, i in enumerate(rows):
        b, e = int(rp[i]), int(rp[i + 1])
        while b < e:
            take = min(e - b, batch - tot)
            win.append((k, b, b + take))
            tot += take
            b += take
            if tot == batch:
                yield win
                win, tot = [], 0
    if win:
        yield win


def _check_split_optimality(m, idx, resid, rp, pm, rows, cols, lam, reg_mode, batch=1_000_000):
    """Worst relative gradient of eq. (SALS) over the listed rows of the last
    mode, the sums over each row's entries taken in windows of `batch`
    entries (so rows of tens of millions of entries fit host memory)."""
    n = m.N - 1
    lens = (rp[rows + 1] - rp[rows]).astype(np.int64)
    assert np.all(lens > 0)
    a = m.factor_block(n, rows, cols)
    g = np.zeros_like(a)
    sc = np.zeros_like(a)
    for win in _pieces(rp, rows, batch):
        J = np.concatenate([pm[b:e] for _, b, e in win]).astype(np.int64)
        seg = np.repeat(np.array([k for k, _, _ in win]), [e - b for _, b, e in win])
        starts = np.concatenate([[0], np.cumsum([e - b for _, b, e in win])[:-1]]).astype(np.int64)
        slots = np.array([k for k, _, _ in win])
        P = _gather_products(m, idx, J, n, cols)
        r = resid[J]
        s = np.abs(r) + (np.abs(P) * np.abs(a[seg])).sum(axis=1)
        np.add.at(g, slots, np.add.reduceat(r[:, None] * P, starts, axis=0))
        np.add.at(sc, slots, np.add.reduceat(np.abs(P) * s[:, None], starts, axis=0))
        del P
    lw = lam * (lens[:, None].astype(np.float64) if reg_mode == 1 else 1.0)
    err = np.abs(g - lw * a) / np.maximum(sc + lw * np.abs(a), 1e-300)
    return float(err.max()), int(rows.shape[0])


def _check_residual(m, idx, x, resid, rng, nsample):
    J = np.unique(rng.integers(0, idx.shape[0], size=nsample))
    P = _gather_products(m, idx, J, -1, None)
    xh = P.sum(axis=1)
    scale = np.abs(x[J]) + np.abs(P).sum(axis=1)
    err_r = float(np.max(np.abs(resid[J] - (x[J] - xh)) / scale))
    err_p = float(np.max(np.abs(m.predict(idx[J]) - xh) / scale))
    return err_r, err_p


def _check_foldin(m, w, F, nreq=200):
    import torch
    from gpu_util import rel_max
    from oracle import oracle as orc
    from paper_1410_5209_amd import tf
    ptr, oidx, vals = synth.make_requests(w.dims, w.R, nreq)
    o = orc.Oracle(w.dims, np.zeros((1, w.N), np.int32), np.zeros(1), w.K, w.lam)
    for n in range(1, w.N):
        o.set_factor(n, F[n])
    d_idx = torch.from_numpy(np.ascontiguousarray(oidx)).cuda()
    d_vals = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
    rows = torch.empty((nreq, w.K), dtype=torch.float64, device="cuda")
    worst = {}
    for method in (tf.TF_FOLDIN_FULL, tf.TF_FOLDIN_CDTF):
        tf.tf_foldin(m.ctx, 0, ptr, d_idx, d_vals, method, 3, rows)
        got = rows.cpu().numpy()
        err = 0.0
        for q in range(nreq):
            sl = slice(ptr[q], ptr[q + 1])
            want = o.foldin_full(0, oidx[sl], vals[sl]) if method == tf.TF_FOLDIN_FULL else \
                o.foldin_cdtf(0, oidx[sl], vals[sl], 3)
            err = max(err, rel_max(got[q], want))
        worst[method] = err
    return worst, int(np.max(np.diff(ptr)))


def _model(w, idx, x, T_in, cands, with_tune=False):
    from paper_1410_5209_amd.model import SparseCP
    m = SparseCP(w.dims, idx, x, w.K, w.lam, precision=w.prec)
    r = m.autotune(T_in, cands, tune_tiles=True)
    return (m, int(r.best_C), r) if with_tune else (m, int(r.best_C))


@pytest.mark.timeout(900)
def test_fullsize_3way():
    """3-way 1M^3, 1e8 uniform entries, K = 100, FP32, C = 10, T_in = 2."""
    w = synth.WORKLOADS["sals-3way-1m-fp32"]
    note(f"fullsize {w.name}: generating {w.nnz} entries")
    idx, x = synth.make_tensor(w)
    note(f"fullsize {w.name}: init + autotune C in [{w.C}]")
    m, C = _model(w, idx, x, w.T_in, [w.C])
    assert C == w.C
    for n in range(w.N):
        note(f"fullsize {w.name}: CSR mode {n}")
        rp, pm = _check_csr(m, idx, n, w.dims[n])
    note(f"fullsize {w.name}: one sweep C={C} T_in={w.T_in}")
    m.sweep(C, w.T_in)
    loss, _ = m.loss()
    resid = m.residual()
    rng = np.random.default_rng(11)
    last = m.col_order()[w.K - C:]
    rows = _rows_to_check(rp, rng, 3000, 0, (0, 0), 10**9)
    worst, nrows = _check_split_optimality(m, idx, resid, rp, pm, rows, last, w.lam, 0)
    note(f"fullsize {w.name}: split optimality over {nrows} rows: {worst:.3g}")
    assert worst <= TOL
    er, ep = _check_residual(m, idx, x, resid, rng, 4000)
    note(f"fullsize {w.name}: residual {er:.3g} predict {ep:.3g}")
    assert er <= TOL and ep <= TOL
    F = m.factors()
    ref = float(np.dot(resid, resid)) + w.lam * sum(float(np.sum(A * A)) for A in F)
    assert abs(loss - ref) <= 1e-10 * ref, (loss, ref)
    note(f"fullsize {w.name}: fold-in of 200 requests")
    worst, mmax = _check_foldin(m, w, F)
    note(f"fullsize {w.name}: fold-in full {worst[0]:.3g} cdtf {worst[1]:.3g} (largest request {mmax})")
    assert worst[0] < 1e-4 and worst[1] < 1e-4
    m.close()


@pytest.mark.timeout(900)
def test_fullsize_3way_bf16():
    """The 3-way workload with BF16 factors and its 1% held-out split (training part)."""
    w = synth.WORKLOADS["sals-3way-1m-bf16"]
    note(f"fullsize {w.name}: generating {w.nnz} entries")
    idx, x = synth.make_tensor(w)[:2]
    note(f"fullsize {w.name}: init + autotune C in [{w.C}]")
    m, C = _model(w, idx, x, w.T_in, [w.C])
    rp, pm = m.csr(w.N - 1)
    note(f"fullsize {w.name}: one sweep C={C} T_in={w.T_in}")
    m.sweep(C, w.T_in)
    resid = m.residual()
    rng = np.random.default_rng(13)
    rows = _rows_to_check(rp, rng, 3000, 0, (0, 0), 10**9)
    worst, nrows = _check_split_optimality(m, idx, resid, rp, pm, rows, m.col_order()[w.K - C:],
                                           w.lam, 0)
    note(f"fullsize {w.name}: split optimality over {nrows} rows: {worst:.3g}")
    assert worst <= 1e-2
    er, ep = _check_residual(m, idx, x, resid, rng, 4000)
    note(f"fullsize {w.name}: residual {er:.3g} predict {ep:.3g}")
    assert er <= TOL and ep <= TOL
    m.close()


@pytest.mark.timeout(900)
def test_fullsize_5way_zipf():
    """5-way 1M^5, 5e8 Zipf(1.0) draws, K = 1000, FP32; C tuned over {16, 32}, T_in = 1.

    The sweep's last split is ragged (K mod C columns), so a further split of C
    columns checks the tuned kernel too."""
    w = synth.WORKLOADS["sals-5way-zipf-fp32"]
    note(f"fullsize {w.name}: generating {w.nnz} draws")
    idx, x = synth.make_tensor(w)
    note(f"fullsize {w.name}: init + autotune C in [16, 32]")
    m, C, tune = _model(w, idx, x, w.T_in, [16, 32], with_tune=True)
    last_mode = w.N - 1
    for n in (0, last_mode):
        note(f"fullsize {w.name}: CSR mode {n}")
        rp, pm = _check_csr(m, idx, n, w.dims[n])
    rng = np.random.default_rng(12)
    # short rows at random, 20 rows split across workgroups, the 3 longest
    # rows of at most 2e6 entries, and the shortest row whose chunks are
    # lengthened so that it has at most 1024 of them (the longest rows hold
    # ~3e7 entries; their sums run the longest FP32 accumulation chains)
    rows = _rows_to_check(rp, rng, 2000, 20, (8192, 50_000), 2_000_000)
    lens = np.diff(rp)
    over = np.flatnonzero(lens > 1024 * int(tune.chunk_nnz[last_mode]))
    if over.size:
        rows = np.unique(np.concatenate([rows, [over[np.argmin(lens[over])]]])).astype(np.int64)
    note(f"fullsize {w.name}: checking rows of up to {int(lens[rows].max())} entries "
         f"(chunk length {int(tune.chunk_nnz[last_mode])})")
    order = m.col_order()
    note(f"fullsize {w.name}: one sweep C={C} T_in={w.T_in}")
    m.sweep(C, w.T_in)
    tail = w.K % C or C
    resid = m.residual()
    worst, nrows = _check_split_optimality(m, idx, resid, rp, pm, rows, order[w.K - tail:], w.lam, 0)
    note(f"fullsize {w.name}: last split ({tail} columns) optimality over {nrows} rows: {worst:.3g}")
    assert worst <= TOL
    er, ep = _check_residual(m, idx, x, resid, rng, 3000)
    note(f"fullsize {w.name}: residual {er:.3g} predict {ep:.3g}")
    assert er <= TOL and ep <= TOL
    cols = order[w.K // 2:w.K // 2 + C]
    note(f"fullsize {w.name}: split of {C} columns")
    m.split(cols, w.T_in)
    del resid
    resid = m.residual()
    worst, nrows = _check_split_optimality(m, idx, resid, rp, pm, rows, cols, w.lam, 0)
    note(f"fullsize {w.name}: {C}-column split optimality over {nrows} rows: {worst:.3g}")
    assert worst <= TOL
    m.close()
