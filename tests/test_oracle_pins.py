"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a stable
sort from numpy (CSR), dense least squares on the stacked system instead of
normal equations + Cholesky (Theorem 1), the scalar closed form of C = 1
(CDTF), eq. (ALS) for C = K, the zero-gradient condition of Theorem 1's
proof, the definition of R recomputed from scratch, the memory theorem
(untouched columns), row independence (Section 3.3), the Eckart-Young
theorem, hand-derived values in exact rational arithmetic, and the published
SplitMix64 outputs.  arXiv:1410.5209 prints no numeric example of the method.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def tiny_problem(seed, dims, nnz, K, dedupe="distinct", first_zero=False):
    idx = synth.tuples(seed, dims, nnz, dedupe=dedupe)
    x = synth.values(seed, dims, idx, 3, 0, 0.1)
    A = synth.factors(seed + 100, dims, K, first_zero=first_zero)
    return idx, x, A


def recon(dims, idx, A, cols=None):
    """sum_k prod_n A_n[i_n, k], vectorised over entries (numpy)."""
    K = A[0].shape[1]
    cols = np.arange(K) if cols is None else np.asarray(cols)
    prod = np.ones((idx.shape[0], len(cols)))
    for n in range(len(dims)):
        prod = prod * A[n][idx[:, n]][:, cols]
    return prod.sum(axis=1)


def make_oracle(dims, idx, x, A, K, lam, reg_mode=0):
    o = orc.Oracle(dims, idx, x, K, lam, reg_mode)
    for n, An in enumerate(A):
        o.set_factor(n, An)
    o.resync()
    return o


def brute_split(dims, idx, x, A, cols, T_in, lam, reg_mode=0):
    """One SALS split by dense least squares: every row of every mode is
    argmin ||P a - t||^2 + lam_i ||a||^2 with t = x - (model of the columns
    outside the split), solved by numpy.linalg.lstsq on [P; sqrt(lam_i) I]."""
    A = [a.copy() for a in A]
    K = A[0].shape[1]
    cols = list(cols)
    rest = [k for k in range(K) if k not in cols]
    t = x - (recon(dims, idx, A, rest) if rest else 0.0)
    for _ in range(T_in):
        for n in range(len(dims)):
            for i in range(dims[n]):
                sel = np.nonzero(idx[:, n] == i)[0]
                if sel.size == 0:
                    A[n][i, cols] = 0.0
                    continue
                P = np.ones((sel.size, len(cols)))
                for l in range(len(dims)):
                    if l != n:
                        P = P * A[l][idx[sel, l]][:, cols]
                lam_i = lam * sel.size if reg_mode else lam
                M = np.vstack([P, np.sqrt(lam_i) * np.eye(len(cols))])
                rhs = np.concatenate([t[sel], np.zeros(len(cols))])
                A[n][i, cols] = np.linalg.lstsq(M, rhs, rcond=None)[0]
    return A


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- P1: CSR

@pytest.mark.parametrize("dedupe", ["distinct", "none"])
def test_csr_is_stable_sort_by_row(dedupe):
    dims = [9, 4, 13]
    idx = synth.tuples(3, dims, 300, dedupe=dedupe)
    x = np.zeros(idx.shape[0])
    o = orc.Oracle(dims, idx, x, 2, 1.0)
    for n in range(3):
        rp, pm = o.get_csr(n)
        want = np.argsort(idx[:, n], kind="stable")
        assert np.array_equal(pm, want)
        cnt = np.bincount(idx[:, n], minlength=dims[n])
        assert np.array_equal(rp, np.concatenate([[0], np.cumsum(cnt)]))


def test_csr_empty_rows_and_single_row():
    dims = [50, 3]
    idx = np.array([[7, 0], [7, 2], [7, 1], [7, 0]], dtype=np.int32)   # duplicates, one row
    o = orc.Oracle(dims, idx, np.ones(4), 1, 1.0)
    rp, pm = o.get_csr(0)
    assert rp[7] == 0 and rp[8] == 4 and rp[-1] == 4 and np.all(rp[:8] == 0)
    assert np.array_equal(pm, [0, 1, 2, 3])
    rp1, pm1 = o.get_csr(1)
    assert np.array_equal(pm1, [0, 3, 2, 1])


# ------------------------------------------------- P2: Theorem 1 / brute force

@pytest.mark.parametrize("N,dims,K,cols,T_in,reg", [
    (3, [6, 5, 7], 4, [1, 3], 1, 0),
    (3, [6, 5, 7], 4, [0, 1, 2, 3], 2, 0),
    (2, [8, 9], 3, [2], 1, 0),
    (4, [4, 5, 3, 6], 5, [4, 0, 2], 2, 1),
    (3, [6, 5, 7], 4, [3, 1, 0], 1, 1),
])
def test_split_equals_dense_least_squares(N, dims, K, cols, T_in, reg):
    idx, x, A = tiny_problem(11 + N, dims, 70, K)
    o = make_oracle(dims, idx, x, A, K, 0.3, reg)
    o.split(cols, T_in)
    want = brute_split(dims, idx, x, A, cols, T_in, 0.3, reg)
    for n in range(N):
        assert rel(o.get_factor(n), want[n]) < 1e-10


def test_split_with_repeated_tuples_equals_dense_least_squares():
    dims = [3, 4, 2]
    idx, x, A = tiny_problem(5, dims, 40, 3, dedupe="none")
    assert len({tuple(t) for t in idx}) < idx.shape[0]          # a multiset (Q8)
    o = make_oracle(dims, idx, x, A, 3, 0.5)
    o.split([0, 2], 2)
    want = brute_split(dims, idx, x, A, [0, 2], 2, 0.5)
    for n in range(3):
        assert rel(o.get_factor(n), want[n]) < 1e-10


def test_last_mode_rows_have_zero_gradient():
    """Theorem 1's proof: after the update, dL/da = 0 for the updated row,
    i.e. sum_j (model_j - x_j) p_j + lambda_i a = 0 over the row's entries."""
    dims = [5, 6, 7]
    K, cols, lam = 4, [0, 2, 3], 0.7
    for reg in (0, 1):
        idx, x, A = tiny_problem(21 + reg, dims, 90, K)
        o = make_oracle(dims, idx, x, A, K, lam, reg)
        o.split(cols, 1)
        F = o.factors()
        r = x - recon(dims, idx, F)
        n = 2
        for i in range(dims[n]):
            sel = np.nonzero(idx[:, n] == i)[0]
            if sel.size == 0:
                continue
            P = np.ones((sel.size, len(cols)))
            for l in (0, 1):
                P = P * F[l][idx[sel, l]][:, cols]
            lam_i = lam * sel.size if reg else lam
            g = -(r[sel] @ P) + lam_i * F[n][i, cols]
            assert np.max(np.abs(g)) < 1e-11 * max(1.0, np.max(np.abs(r[sel] @ P)))


def test_row_update_matches_dense_least_squares_on_current_state():
    dims = [6, 5, 7]
    K, cols = 4, [2, 0]
    idx, x, A = tiny_problem(31, dims, 80, K)
    o = make_oracle(dims, idx, x, A, K, 0.2)
    want = brute_split(dims, idx, x, A, cols, 1, 0.2)        # mode 0 is updated first
    for i in range(dims[0]):
        assert rel(o.row_update(0, i, cols), want[0][i, cols]) < 1e-10


@pytest.mark.parametrize("reg", [0, 1])
def test_sweep_walks_the_order_in_blocks_of_dense_least_squares_splits(reg):
    """Algorithm 1's outer iteration: the column order is taken in ceil(K/C)
    blocks of C columns, the last block shorter when C does not divide K
    (reading Q4), and every block is one split.  K = 7, C = 3 gives blocks of
    3, 3 and 1 columns of a non-identity order; each is checked against the
    dense least-squares split applied to the factors the previous block left
    (its target x minus the model of the columns outside the block, recomputed
    from scratch, so the residual the oracle carries between splits is pinned
    too).  Over two sweeps, T_in = 2."""
    dims = [6, 5, 7]
    K, C, T_in = 7, 3, 2
    lam = 0.02 if reg else 0.35    # weighted: lambda_i = lambda |Omega_i| (~15 entries a row)
    order = [4, 0, 6, 2, 5, 1, 3]
    idx, x, A = tiny_problem(91 + reg, dims, 110, K)
    o = make_oracle(dims, idx, x, A, K, lam, reg)
    want = [a.copy() for a in A]
    for _ in range(2):
        o.sweep(C, T_in, order)
        blocks = [order[s:s + C] for s in range(0, K, C)]
        assert [len(b) for b in blocks] == [3, 3, 1]
        for cols in blocks:
            want = brute_split(dims, idx, x, want, cols, T_in, lam, reg)
        for n in range(3):
            assert np.max(np.abs(want[n])) > 0.05              # not shrunk to zero
            assert rel(o.get_factor(n), want[n]) < 1e-9, n
        assert np.max(np.abs(o.residual() - (x - recon(dims, idx, want)))) < 1e-9 * np.max(np.abs(x))


# ------------------------------------------------------- P3: CDTF closed form

def test_cdtf_equals_scalar_closed_form():
    """C = 1: a = sum_j rhat_j p_j / (lambda_i + sum_j p_j^2)."""
    dims = [7, 6, 5]
    K, lam = 3, 0.4
    idx, x, A = tiny_problem(41, dims, 90, K)
    o = make_oracle(dims, idx, x, A, K, lam)
    k = 1
    rhat = x - recon(dims, idx, A, [0, 2])
    for n in range(3):
        for i in range(dims[n]):
            sel = np.nonzero(idx[:, n] == i)[0]
            p = np.ones(sel.size)
            for l in range(3):
                if l != n:
                    p = p * A[l][idx[sel, l], k]
            want = (rhat[sel] @ p) / (lam + p @ p) if sel.size else 0.0
            got = o.row_update(n, i, [k])[0]
            assert abs(got - want) <= 1e-13 * max(1.0, abs(want))


# ------------------------------------------------------------ P4: C = K is ALS

def test_full_split_is_als():
    """C = K, T_in = 1: every row solves eq. (ALS) with c built from x."""
    dims = [5, 6, 4]
    K, lam = 3, 0.25
    idx, x, A = tiny_problem(51, dims, 70, K)
    o = make_oracle(dims, idx, x, A, K, lam)
    o.sweep(K, 1)
    F = [a.copy() for a in A]
    for n in range(3):
        for i in range(dims[n]):
            sel = np.nonzero(idx[:, n] == i)[0]
            if sel.size == 0:
                F[n][i] = 0.0
                continue
            P = np.ones((sel.size, K))
            for l in range(3):
                if l != n:
                    P = P * F[l][idx[sel, l]]
            B = P.T @ P + lam * np.eye(K)
            F[n][i] = np.linalg.solve(B, P.T @ x[sel])
    for n in range(3):
        assert rel(o.get_factor(n), F[n]) < 1e-11


# ----------------------------------------------------- P5: monotone loss, P6, P7

@pytest.mark.parametrize("reg", [0, 1])
def test_loss_never_increases_and_residual_is_exact(reg):
    dims = [20, 15, 12]
    K, lam = 5, 0.1
    idx, x, A = tiny_problem(61 + reg, dims, 600, K, first_zero=True)
    o = make_oracle(dims, idx, x, A, K, lam, reg)
    prev = o.loss()[0]
    for sweep in range(3):
        order = synth.column_order(synth.SEED_ORDER, sweep, K)
        for s in range(0, K, 2):
            cols = order[s:s + 2]
            before = [o.get_factor(n) for n in range(3)]
            o.split(cols, 2)
            cur = o.loss()[0]
            assert cur <= prev * (1 + 1e-12)
            prev = cur
            F = o.factors()
            # P6: the maintained residual is x - recon from scratch
            assert np.max(np.abs(o.residual() - (x - recon(dims, idx, F)))) < 1e-10 * np.max(np.abs(x))
            # P7: columns outside the split are bit-unchanged
            other = [k for k in range(K) if k not in set(cols.tolist())]
            for n in range(3):
                assert np.array_equal(F[n][:, other], before[n][:, other])


def test_loss_hand_example():
    """eq. (TF) on a 2x2 example worked by hand in exact arithmetic:
    A1 = [[1],[2]], A2 = [[3],[1/2]], observed (0,0)=4, (1,1)=0, (0,1)=1.
    Model 3, 1, 1/2; residuals 1, -1, 1/2; sum r^2 = 9/4.
    Plain: lambda (1+4+9+1/4); weighted: lambda (2*1 + 1*4 + 1*9 + 2*1/4)."""
    lam = Fraction(1, 10)
    idx = np.array([[0, 0], [1, 1], [0, 1]], dtype=np.int32)
    x = np.array([4.0, 0.0, 1.0])
    for reg, want in ((0, Fraction(9, 4) + lam * Fraction(57, 4)),
                      (1, Fraction(9, 4) + lam * Fraction(31, 2))):
        o = orc.Oracle([2, 2], idx, x, 1, float(lam), reg)
        o.set_factor(0, np.array([[1.0], [2.0]]))
        o.set_factor(1, np.array([[3.0], [0.5]]))
        o.resync()
        loss, rmse = o.loss()
        assert abs(loss - float(want)) < 1e-15
        assert abs(rmse - np.sqrt(9 / 4 / 3)) < 1e-15


def test_cdtf_hand_example():
    """Worked C = 1 update on the same example, mode 0, row 0, column 0:
    entries (0,0) and (0,1); p = (3, 1/2); rhat = r + a*p = (1+3, 1/2+1/2) = (4, 1);
    a = (4*3 + 1*1/2) / (lambda + 9 + 1/4) with lambda = 1/10 -> 125/93."""
    idx = np.array([[0, 0], [1, 1], [0, 1]], dtype=np.int32)
    o = orc.Oracle([2, 2], idx, np.array([4.0, 0.0, 1.0]), 1, 0.1)
    o.set_factor(0, np.array([[1.0], [2.0]]))
    o.set_factor(1, np.array([[3.0], [0.5]]))
    o.resync()
    got = o.row_update(0, 0, [0])[0]
    assert abs(got - float(Fraction(25, 2) / Fraction(187, 20))) < 1e-15


# ---------------------------------------------------- P8: row independence

def test_row_relabeling_is_bit_invariant():
    dims = [11, 9, 8]
    K = 4
    idx, x, A = tiny_problem(71, dims, 200, K)
    o1 = make_oracle(dims, idx, x, A, K, 0.2)
    o1.sweep(2, 2)
    perms = [synth.permutation(9, 40 + n, d) for n, d in enumerate(dims)]   # new = perm[old]
    idx2 = np.stack([perms[n][idx[:, n]] for n in range(3)], axis=1)
    A2 = []
    for n in range(3):
        B = np.empty_like(A[n])
        B[perms[n]] = A[n]
        A2.append(B)
    o2 = make_oracle(dims, idx2, x, A2, K, 0.2)
    o2.sweep(2, 2)
    for n in range(3):
        assert np.array_equal(o2.get_factor(n)[perms[n]], o1.get_factor(n))


def test_entry_order_changes_only_rounding():
    dims = [11, 9, 8]
    K = 4
    idx, x, A = tiny_problem(72, dims, 200, K)
    o1 = make_oracle(dims, idx, x, A, K, 0.2)
    o1.sweep(3, 1)
    sh = synth.permutation(9, 60, idx.shape[0])
    o2 = make_oracle(dims, idx[sh], x[sh], A, K, 0.2)
    o2.sweep(3, 1)
    for n in range(3):
        assert rel(o2.get_factor(n), o1.get_factor(n)) < 1e-12


# --------------------------------------------------------- P9: Eckart-Young

def test_fully_observed_matrix_reaches_eckart_young():
    m, n_, r = 12, 9, 3
    g = np.random.default_rng(0)
    X = g.standard_normal((m, r)) @ g.standard_normal((r, n_)) + 0.05 * g.standard_normal((m, n_))
    ii, jj = np.meshgrid(np.arange(m), np.arange(n_), indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel()], axis=1).astype(np.int32)
    x = X.ravel()
    lam = 1e-9
    o = orc.Oracle([m, n_], idx, x, r, lam)
    o.set_factor(0, np.zeros((m, r)))
    o.set_factor(1, g.random((n_, r)))
    o.resync()
    for _ in range(3000):
        o.sweep(r, 1)
    sv = np.linalg.svd(X, compute_uv=False)
    want = float(np.sum(sv[r:] ** 2))
    F = o.factors()
    se = float(np.sum((x - recon([m, n_], idx, F)) ** 2))
    assert abs(se - want) <= 1e-6 * want


# ----------------------------------------------------------------- fold-in

def test_foldin_full_rank_is_dense_least_squares():
    dims = [6, 9, 7]
    K, lam = 4, 0.3
    idx, x, A = tiny_problem(81, dims, 120, K)
    for reg in (0, 1):
        o = make_oracle(dims, idx, x, A, K, lam, reg)
        g = np.random.default_rng(1)
        m = 15
        oidx = np.stack([g.integers(0, dims[1], m), g.integers(0, dims[2], m)], 1).astype(np.int32)
        v = g.standard_normal(m)
        P = A[1][oidx[:, 0]] * A[2][oidx[:, 1]]
        lam_i = lam * m if reg else lam
        M = np.vstack([P, np.sqrt(lam_i) * np.eye(K)])
        want = np.linalg.lstsq(M, np.concatenate([v, np.zeros(K)]), rcond=None)[0]
        assert rel(o.foldin_full(0, oidx, v), want) < 1e-10
        assert np.all(o.foldin_full(0, oidx[:0], v[:0]) == 0.0)


def test_foldin_cdtf_converges_to_full_rank_and_one_column_closed_form():
    dims = [6, 9, 7]
    K, lam = 3, 0.3
    idx, x, A = tiny_problem(82, dims, 120, K)
    o = make_oracle(dims, idx, x, A, K, lam)
    g = np.random.default_rng(2)
    m = 10
    oidx = np.stack([g.integers(0, dims[0], m), g.integers(0, dims[2], m)], 1).astype(np.int32)
    v = g.standard_normal(m)
    full = o.foldin_full(1, oidx, v)
    # coordinate descent on a strictly convex quadratic converges to its minimiser
    assert rel(o.foldin_cdtf(1, oidx, v, 400), full) < 1e-9
    # one sweep, first column: a_0 = sum x p_0 / (lambda + sum p_0^2) (a starts at 0)
    p0 = A[0][oidx[:, 0], 0] * A[2][oidx[:, 1], 0]
    a1 = o.foldin_cdtf(1, oidx, v, 1)
    assert abs(a1[0] - (v @ p0) / (lam + p0 @ p0)) < 1e-13


# ----------------------------------------------------------- predict

def test_predict_hand_example():
    idx = np.array([[0, 0], [1, 1]], dtype=np.int32)
    o = orc.Oracle([2, 2], idx, np.zeros(2), 2, 1.0)
    o.set_factor(0, np.array([[1.0, 2.0], [0.5, -1.0]]))
    o.set_factor(1, np.array([[3.0, 4.0], [2.0, 0.25]]))
    got = o.predict(np.array([[0, 0], [1, 1], [0, 1], [1, 0]]))
    assert np.array_equal(got, [1 * 3 + 2 * 4, 0.5 * 2 - 1 * 0.25, 1 * 2 + 2 * 0.25, 0.5 * 3 - 4])


# ------------------------------------------------------- validation, Q6, Q7

def test_invalid_inputs_rejected():
    idx = np.array([[0, 0]], dtype=np.int32)
    with pytest.raises(orc.OracleError):
        orc.Oracle([2, 2], idx, np.ones(1), 1, 0.0)            # Q7: lambda must be > 0
    with pytest.raises(orc.OracleError):
        orc.Oracle([2, 2], np.array([[2, 0]], dtype=np.int32), np.ones(1), 1, 1.0)
    with pytest.raises(orc.OracleError):
        orc.Oracle([2, 2], idx, np.array([np.nan]), 1, 1.0)


def test_empty_row_set_to_zero():
    idx = np.array([[0, 0], [0, 1]], dtype=np.int32)
    for reg in (0, 1):
        o = orc.Oracle([3, 2], idx, np.array([1.0, 2.0]), 2, 0.5, reg)
        o.set_factor(0, np.full((3, 2), 0.7))
        o.set_factor(1, np.full((2, 2), 0.3))
        o.resync()
        o.split([0, 1], 1)
        F = o.get_factor(0)
        assert np.all(F[1:] == 0.0) and np.all(F[0] != 0.0)


# -------------------------------------------------------------- RNG pin

def _golden_splitmix():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                s, t, v = line.split()
                rows.append((int(s), int(t), int(v)))
    return rows


def test_splitmix64_published_outputs():
    for s, t, v in _golden_splitmix():
        assert orc.splitmix64(s, t) == v


def test_library_init_rule_uses_splitmix_counters():
    rows = _golden_splitmix()
    seed = rows[0][0]
    dims, K = [2, 3], 4
    o = orc.Oracle(dims, np.array([[0, 0]], dtype=np.int32), np.ones(1), K, 1.0)
    o.init_factors(seed, first_factor_zero=False)
    A0 = o.get_factor(0)
    for s, t, v in rows:            # counters 1..5 are entries 0..4 of factor 0 (row-major)
        i, k = divmod(t - 1, K)
        assert A0[i, k] == (v >> 11) * 2.0 ** -53 / 2.0
    o.init_factors(seed, first_factor_zero=True)
    assert np.all(o.get_factor(0) == 0.0)
    A1 = o.get_factor(1)
    assert np.all((A1 >= 0) & (A1 < 0.5))
    assert A1[0, 0] == (orc.splitmix64(seed, 1 + dims[0] * K) >> 11) * 2.0 ** -53 / 2.0


def test_random_column_order_is_a_uniform_permutation_from_splitmix():
    """The random column order (Algorithm 1 draws the columns of each split
    without replacement): a permutation of 0..K-1 for every sweep; for K = 2
    the one step swaps unless the top bit of SplitMix64 output 2^62 + 2t + 1 is set
    (pinned by the published outputs above); for K = 3 all six orders appear
    about equally often (a shuffle whose index range missed position i
    would give only the two cyclic ones)."""
    for K in (1, 2, 7, 100):
        for t in range(5):
            order = orc.column_order(12345, t, K)
            assert sorted(order.tolist()) == list(range(K))
    for t in range(64):   # j = top bit; j = 1 leaves position 1 in place
        top = orc.splitmix64(99, (1 << 62) + 2 * t + 1) >> 63
        assert orc.column_order(99, t, 2).tolist() == ([0, 1] if top else [1, 0])
    counts = {}
    n = 6000
    for t in range(n):
        key = tuple(orc.column_order(7, t, 3).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    chi2 = sum((c - n / 6) ** 2 / (n / 6) for c in counts.values())
    assert chi2 < 25.0   # 5 degrees of freedom: p < 1e-4 beyond this
