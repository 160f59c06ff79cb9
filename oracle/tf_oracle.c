/*
 * tf_oracle.c -- plain FP64 CPU oracle for the SALS / CDTF row-update path.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * GPU path; the two meet only through the seeded inputs of the synth module.
 *
 * What it computes, and where the paper defines it
 * (K. Shin, U Kang, "Distributed Methods for High-dimensional and Large-scale
 * Tensor Factorization", arXiv:1410.5209):
 *
 *   loss ............ Definition 1, eq. (TF): squared error over the observed
 *                     entries plus lambda times the squared Frobenius norms.
 *   residual ........ Section 3.1: r = x - sum_k prod_n a^(n)_{i_n k}.
 *   split ........... Algorithm 1 (serial SALS): pick C columns, form R-hat,
 *                     T_in inner iterations over the modes, every row of the
 *                     mode updated by eq. (SALS), then R updated by
 *                     eq. (SALS_R).
 *   row update ...... eq. (SALS) with B and c as defined beside it; Theorem 1
 *                     shows it is the exact minimiser; the text after the
 *                     theorem solves it with a Cholesky factorisation.
 *   CDTF ............ SALS with C = 1 (end of Section 3.1).
 *   ALS ............. eq. (ALS); equals SALS with C = K and T_in = 1.
 *   weighted lambda . Section 5.1.3 (ALS-WR weighting lambda * |Omega_i|).
 *   fold-in ......... eq. (ALS) for one new row (full rank) and the CDTF
 *                     coordinate update for one new row; a use of the row
 *                     update that the paper does not itself make.
 *
 * Readings where the paper is silent (numbered as in the design notes):
 *   Q3  columns are taken in the order the caller passes; a sweep walks that
 *       order in blocks of C, the last block shorter when C does not divide K.
 *   Q6  a row with no observed entries is set to zero.
 *   Q7  lambda must be positive.
 *   Q8  a repeated index tuple is one more loss term (multiset).
 *   Q14 all sums run sequentially: entries of a row in CSR order (stable,
 *       input order inside a row), columns ascending, modes ascending.
 *
 * Nothing here is blocked, fused or reordered beyond what the definitions
 * state.  Rows of one mode are independent given the other factors
 * (Section 3.3), so the row loop of a mode may run on several threads; every
 * other loop, and every reduction, is sequential.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_NOMEM 2
#define OR_E_NUMERIC 4

typedef struct or_ctx {
    int N;
    int64_t dims[8];
    int64_t nnz;
    int32_t *idx;      /* nnz x N, row-major, 0-based, input order */
    double *x;         /* nnz observed values, input order */
    int K;
    double lambda;
    int reg_mode;      /* 0: lambda (eq. TF); 1: lambda * |Omega_i^(n)| */
    double *A[8];      /* factor n: dims[n] x K, row-major */
    double *r;         /* residual, input order (Section 3.1) */
    int64_t *rowptr[8];/* mode-n CSR: dims[n] + 1 offsets */
    int32_t *perm[8];  /* mode-n CSR: entry ids, stable inside a row */
    int64_t bad_row;   /* row of the last non-positive pivot, or -1 */
    int bad_mode;
} or_ctx;

/* ---------------------------------------------------------------------- */
/* CSR of one mode: the sets Omega^(n)_{i_n} of Table 1, listed row by row.
 * Counting sort; entries keep their input order inside a row.            */
static int build_csr(or_ctx *c, int n)
{
    int64_t I = c->dims[n];
    int64_t *rp = (int64_t *)calloc((size_t)I + 1, sizeof(int64_t));
    int32_t *pm = (int32_t *)malloc((size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)(I > 0 ? I : 1) * sizeof(int64_t));
    if (!rp || !pm || !fill) { free(rp); free(pm); free(fill); return OR_E_NOMEM; }
    for (int64_t j = 0; j < c->nnz; ++j) rp[c->idx[j * c->N + n] + 1] += 1;
    for (int64_t i = 0; i < I; ++i) rp[i + 1] += rp[i];
    for (int64_t i = 0; i < I; ++i) fill[i] = rp[i];
    for (int64_t j = 0; j < c->nnz; ++j) {
        int64_t i = c->idx[j * c->N + n];
        pm[fill[i]] = (int32_t)j;
        fill[i] += 1;
    }
    free(fill);
    c->rowptr[n] = rp;
    c->perm[n] = pm;
    return OR_OK;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    free(c->idx); free(c->x); free(c->r);
    for (int n = 0; n < 8; ++n) { free(c->A[n]); free(c->rowptr[n]); free(c->perm[n]); }
    free(c);
}

/* Validation follows the same rules as the library (Q7: lambda > 0). */
int or_create(int N, const int64_t *dims, int64_t nnz, const int32_t *idx,
              const double *vals, int K, double lambda, int reg_mode, or_ctx **out)
{
    *out = NULL;
    if (N < 2 || N > 8 || nnz < 0 || K < 1 || !(lambda > 0.0) || (reg_mode != 0 && reg_mode != 1))
        return OR_E_INVALID;
    for (int n = 0; n < N; ++n) if (dims[n] < 1) return OR_E_INVALID;
    for (int64_t j = 0; j < nnz; ++j) {
        if (!isfinite(vals[j])) return OR_E_INVALID;
        for (int n = 0; n < N; ++n) {
            int32_t v = idx[j * N + n];
            if (v < 0 || v >= dims[n]) return OR_E_INVALID;
        }
    }
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    if (!c) return OR_E_NOMEM;
    c->N = N; c->nnz = nnz; c->K = K; c->lambda = lambda; c->reg_mode = reg_mode;
    c->bad_row = -1; c->bad_mode = -1;
    for (int n = 0; n < N; ++n) c->dims[n] = dims[n];
    size_t ne = (size_t)(nnz > 0 ? nnz : 1);
    c->idx = (int32_t *)malloc(ne * (size_t)N * sizeof(int32_t));
    c->x = (double *)malloc(ne * sizeof(double));
    c->r = (double *)malloc(ne * sizeof(double));
    if (!c->idx || !c->x || !c->r) { or_destroy(c); return OR_E_NOMEM; }
    memcpy(c->idx, idx, (size_t)nnz * (size_t)N * sizeof(int32_t));
    memcpy(c->x, vals, (size_t)nnz * sizeof(double));
    for (int n = 0; n < N; ++n) {
        c->A[n] = (double *)calloc((size_t)dims[n] * (size_t)K, sizeof(double));
        if (!c->A[n]) { or_destroy(c); return OR_E_NOMEM; }
        if (build_csr(c, n) != OR_OK) { or_destroy(c); return OR_E_NOMEM; }
    }
    /* All factors start at zero, so R = X (Section 3.1). */
    memcpy(c->r, c->x, (size_t)nnz * sizeof(double));
    *out = c;
    return OR_OK;
}

void or_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_set_factor(or_ctx *c, int n, const double *h)
{
    if (n < 0 || n >= c->N) return OR_E_INVALID;
    memcpy(c->A[n], h, (size_t)c->dims[n] * (size_t)c->K * sizeof(double));
    return OR_OK;
}

int or_get_factor(const or_ctx *c, int n, double *h)
{
    if (n < 0 || n >= c->N) return OR_E_INVALID;
    memcpy(h, c->A[n], (size_t)c->dims[n] * (size_t)c->K * sizeof(double));
    return OR_OK;
}

int or_get_csr(const or_ctx *c, int n, int64_t *rowptr, int32_t *perm)
{
    if (n < 0 || n >= c->N) return OR_E_INVALID;
    memcpy(rowptr, c->rowptr[n], (size_t)(c->dims[n] + 1) * sizeof(int64_t));
    memcpy(perm, c->perm[n], (size_t)c->nnz * sizeof(int32_t));
    return OR_OK;
}

void or_get_residual(const or_ctx *c, double *h)
{
    memcpy(h, c->r, (size_t)c->nnz * sizeof(double));
}

void or_set_residual(or_ctx *c, const double *h)
{
    memcpy(c->r, h, (size_t)c->nnz * sizeof(double));
}

/* Model value of entry j restricted to a column list:
 * sum over the listed k of prod_n a^(n)_{i_n k} (modes ascending). */
static double model_cols(const or_ctx *c, int64_t j, int ncols, const int32_t *cols)
{
    double s = 0.0;
    for (int q = 0; q < ncols; ++q) {
        double prod = 1.0;
        for (int n = 0; n < c->N; ++n)
            prod *= c->A[n][(int64_t)c->idx[j * c->N + n] * c->K + cols[q]];
        s += prod;
    }
    return s;
}

/* r = x - sum_{k=1..K} prod_n a^(n)_{i_n k}  (definition of R, Section 3.1). */
void or_resync(or_ctx *c)
{
    int32_t *all = (int32_t *)malloc((size_t)c->K * sizeof(int32_t));
    for (int k = 0; k < c->K; ++k) all[k] = k;
    for (int64_t j = 0; j < c->nnz; ++j) c->r[j] = c->x[j] - model_cols(c, j, c->K, all);
    free(all);
}

/* Cholesky solve of (M) a = b for a symmetric positive-definite C x C matrix
 * given as a full row-major array (text after Theorem 1).  No pivoting.
 * Returns 0, or -1 when a pivot is not positive. */
static int cholesky_solve(int C, double *M, const double *b, double *a)
{
    /* M = L L^T, L stored in the lower triangle of M */
    for (int j = 0; j < C; ++j) {
        double d = M[j * C + j];
        for (int k = 0; k < j; ++k) d -= M[j * C + k] * M[j * C + k];
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        M[j * C + j] = ljj;
        for (int i = j + 1; i < C; ++i) {
            double s = M[i * C + j];
            for (int k = 0; k < j; ++k) s -= M[i * C + k] * M[j * C + k];
            M[i * C + j] = s / ljj;
        }
    }
    /* L y = b */
    double *y = (double *)malloc((size_t)C * sizeof(double));
    for (int i = 0; i < C; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= M[i * C + k] * y[k];
        y[i] = s / M[i * C + i];
    }
    /* L^T a = y */
    for (int i = C - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < C; ++k) s -= M[k * C + i] * a[k];
        a[i] = s / M[i * C + i];
    }
    free(y);
    return 0;
}

/* The update of one row by eq. (SALS): a = (B + lambda_i I_C)^{-1} c with
 *   B[c1][c2] = sum_{j in Omega_i} p_j[c1] p_j[c2],
 *   c[c]      = sum_{j in Omega_i} rhat_j p_j[c],
 *   p_j[c]    = prod_{l != n} a^(l)_{i_l k_c}.
 * Reads the other modes only; writes nothing.  Q6: an empty row gives 0. */
static int row_solve(const or_ctx *c, int n, int64_t i, int ncols, const int32_t *cols,
                     const double *rhat, const double *rhat_row, double *a_out)
{
    int C = ncols;
    int64_t beg = c->rowptr[n][i], end = c->rowptr[n][i + 1];
    if (end == beg) {
        for (int q = 0; q < C; ++q) a_out[q] = 0.0;
        return 0;
    }
    double *M = (double *)calloc((size_t)C * C, sizeof(double));
    double *rhs = (double *)calloc((size_t)C, sizeof(double));
    double *p = (double *)malloc((size_t)C * sizeof(double));
    for (int64_t q = beg; q < end; ++q) {
        int64_t j = c->perm[n][q];
        for (int cc = 0; cc < C; ++cc) {
            double prod = 1.0;
            for (int l = 0; l < c->N; ++l) {
                if (l == n) continue;
                prod *= c->A[l][(int64_t)c->idx[j * c->N + l] * c->K + cols[cc]];
            }
            p[cc] = prod;
        }
        /* rhat by entry id, or (single-row use) by position inside the row */
        double rh = rhat_row ? rhat_row[q - beg] : rhat[j];
        for (int c1 = 0; c1 < C; ++c1) {
            for (int c2 = 0; c2 < C; ++c2) M[c1 * C + c2] += p[c1] * p[c2];
            rhs[c1] += rh * p[c1];
        }
    }
    double lam = c->reg_mode ? c->lambda * (double)(end - beg) : c->lambda;
    for (int q = 0; q < C; ++q) M[q * C + q] += lam;
    int rc = cholesky_solve(C, M, rhs, a_out);
    free(M); free(rhs); free(p);
    return rc;
}

static int check_cols(const or_ctx *c, int ncols, const int32_t *cols)
{
    if (ncols < 1 || ncols > c->K) return OR_E_INVALID;
    for (int q = 0; q < ncols; ++q) {
        if (cols[q] < 0 || cols[q] >= c->K) return OR_E_INVALID;
        for (int s = 0; s < q; ++s) if (cols[s] == cols[q]) return OR_E_INVALID;
    }
    return OR_OK;
}

/* R-hat of a split (Section 3.1): the residual with the split's columns'
 * current contribution added back, i.e. x minus the model of every column
 * outside the split. */
static void form_rhat(const or_ctx *c, int ncols, const int32_t *cols, double *rhat)
{
    for (int64_t j = 0; j < c->nnz; ++j) rhat[j] = c->r[j] + model_cols(c, j, ncols, cols);
}

/* Every row of mode n replaced by its eq. (SALS) minimiser against rhat.
 * Rows of one mode read only the other modes (Section 3.3), so they are
 * independent.  A row whose Cholesky meets a non-positive pivot keeps its
 * value; the smallest such row is returned (-1 if none). */
static int64_t update_mode(or_ctx *c, int n, int ncols, const int32_t *cols, const double *rhat)
{
    int64_t I = c->dims[n];
    int64_t bad = -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < I; ++i) {
        double a[64];
        double *ap = ncols <= 64 ? a : (double *)malloc((size_t)ncols * sizeof(double));
        if (row_solve(c, n, i, ncols, cols, rhat, NULL, ap) != 0) {
#pragma omp critical
            { if (bad < 0 || i < bad) bad = i; }
        } else {
            for (int q = 0; q < ncols; ++q) c->A[n][i * c->K + cols[q]] = ap[q];
        }
        if (ap != a) free(ap);
    }
    return bad;
}

/* R after a split, eq. (SALS_R): rhat minus the split's columns' new
 * contribution. */
static void residual_after_split(or_ctx *c, int ncols, const int32_t *cols, const double *rhat)
{
    for (int64_t j = 0; j < c->nnz; ++j) c->r[j] = rhat[j] - model_cols(c, j, ncols, cols);
}

/* One split of serial SALS (Algorithm 1) on the columns cols[0..ncols):
 * R-hat, then T_in inner iterations each replacing the rows of modes
 * 1..N in turn, then R by eq. (SALS_R).  A non-positive pivot ends the
 * inner iterations after the mode where it happened (that mode's other rows
 * are updated); R is still brought up to date, so the state stays
 * consistent. */
int or_split(or_ctx *c, int ncols, const int32_t *cols, int T_in)
{
    if (check_cols(c, ncols, cols) != OR_OK || T_in < 1) return OR_E_INVALID;
    double *rhat = (double *)malloc((size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(double));
    if (!rhat) return OR_E_NOMEM;
    form_rhat(c, ncols, cols, rhat);
    int status = OR_OK;
    for (int it = 0; it < T_in && status == OR_OK; ++it) {
        for (int n = 0; n < c->N && status == OR_OK; ++n) {
            int64_t bad = update_mode(c, n, ncols, cols, rhat);
            if (bad >= 0) { c->bad_row = bad; c->bad_mode = n; status = OR_E_NUMERIC; }
        }
    }
    residual_after_split(c, ncols, cols, rhat);
    free(rhat);
    return status;
}

/* Block s of an outer iteration over K columns in blocks of C (reading Q4:
 * ceil(K/C) blocks, the last one shorter when C does not divide K). */
static int block_width(int K, int C, int s)
{
    int start = s * C;
    return K - start < C ? K - start : C;
}

/* One outer iteration of serial SALS (Algorithm 1): the column order
 * `order` (a permutation of 0..K-1) taken block by block, one split per
 * block.  Stops at the first split that meets a non-positive pivot. */
int or_sweep(or_ctx *c, int C, int T_in, const int32_t *order)
{
    if (C < 1 || C > c->K || T_in < 1) return OR_E_INVALID;
    if (check_cols(c, c->K, order) != OR_OK) return OR_E_INVALID;
    int nblocks = (c->K + C - 1) / C;
    for (int s = 0; s < nblocks; ++s) {
        int rc = or_split(c, block_width(c->K, C, s), order + (int64_t)s * C, T_in);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* Row update evaluated on the current state without changing it: the value
 * eq. (SALS) gives row i of mode n when R-hat is formed for `cols` from the
 * current residual.  Used to check single rows of large runs. */
int or_row_update(const or_ctx *c, int n, int64_t i, int ncols, const int32_t *cols, double *a_out)
{
    if (n < 0 || n >= c->N || i < 0 || i >= c->dims[n]) return OR_E_INVALID;
    if (check_cols(c, ncols, cols) != OR_OK) return OR_E_INVALID;
    int64_t beg = c->rowptr[n][i], end = c->rowptr[n][i + 1];
    /* rhat over the row's entries only, by position inside the row */
    double *rh = (double *)malloc((size_t)(end > beg ? end - beg : 1) * sizeof(double));
    for (int64_t q = beg; q < end; ++q) {
        int64_t j = c->perm[n][q];
        rh[q - beg] = c->r[j] + model_cols(c, j, ncols, cols);
    }
    int rc = row_solve(c, n, i, ncols, cols, NULL, rh, a_out);
    free(rh);
    return rc == 0 ? OR_OK : OR_E_NUMERIC;
}

int64_t or_bad_row(const or_ctx *c) { return c->bad_row; }
int or_bad_mode(const or_ctx *c) { return c->bad_mode; }

/* eq. (TF): sum r^2 + lambda * sum_n ||A^(n)||_F^2; in weighted mode every
 * row's squared norm is weighted by |Omega_i^(n)|.  Sequential sums. */
void or_loss(const or_ctx *c, double *loss, double *rmse)
{
    double se = 0.0;
    for (int64_t j = 0; j < c->nnz; ++j) se += c->r[j] * c->r[j];
    double reg = 0.0;
    for (int n = 0; n < c->N; ++n) {
        for (int64_t i = 0; i < c->dims[n]; ++i) {
            double w = c->reg_mode ? (double)(c->rowptr[n][i + 1] - c->rowptr[n][i]) : 1.0;
            double rs = 0.0;
            for (int k = 0; k < c->K; ++k) rs += c->A[n][i * c->K + k] * c->A[n][i * c->K + k];
            reg += w * rs;
        }
    }
    *loss = se + c->lambda * reg;
    *rmse = c->nnz > 0 ? sqrt(se / (double)c->nnz) : 0.0;
}

/* x-hat = sum_k prod_n a^(n)_{i_n k} for m query tuples (m x N). */
int or_predict(const or_ctx *c, int64_t m, const int32_t *q, double *out)
{
    for (int64_t t = 0; t < m; ++t)
        for (int n = 0; n < c->N; ++n)
            if (q[t * c->N + n] < 0 || q[t * c->N + n] >= c->dims[n]) return OR_E_INVALID;
    for (int64_t t = 0; t < m; ++t) {
        double s = 0.0;
        for (int k = 0; k < c->K; ++k) {
            double prod = 1.0;
            for (int n = 0; n < c->N; ++n) prod *= c->A[n][(int64_t)q[t * c->N + n] * c->K + k];
            s += prod;
        }
        out[t] = s;
    }
    return OR_OK;
}

/* p_j[k] for a fold-in request: product over the modes other than `mode`
 * of the resident factor rows; `oidx` lists those modes ascending. */
static double fold_p(const or_ctx *c, int mode, const int32_t *oidx, int64_t j, int k)
{
    double prod = 1.0;
    int t = 0;
    for (int l = 0; l < c->N; ++l) {
        if (l == mode) continue;
        prod *= c->A[l][(int64_t)oidx[j * (c->N - 1) + t] * c->K + k];
        t += 1;
    }
    return prod;
}

static int check_fold(const or_ctx *c, int mode, int64_t m, const int32_t *oidx, const double *vals)
{
    if (mode < 0 || mode >= c->N || m < 0) return OR_E_INVALID;
    for (int64_t j = 0; j < m; ++j) {
        if (!isfinite(vals[j])) return OR_E_INVALID;
        int t = 0;
        for (int l = 0; l < c->N; ++l) {
            if (l == mode) continue;
            int32_t v = oidx[j * (c->N - 1) + t];
            if (v < 0 || v >= c->dims[l]) return OR_E_INVALID;
            t += 1;
        }
    }
    return OR_OK;
}

/* Full-rank fold-in of one new row of mode `mode`: eq. (ALS) with c built
 * from the request's values, a = (B + lambda_i I_K)^{-1} c. */
int or_foldin_full(const or_ctx *c, int mode, int64_t m, const int32_t *oidx,
                   const double *vals, double *row_out)
{
    if (check_fold(c, mode, m, oidx, vals) != OR_OK) return OR_E_INVALID;
    int K = c->K;
    if (m == 0) { for (int k = 0; k < K; ++k) row_out[k] = 0.0; return OR_OK; }
    double *M = (double *)calloc((size_t)K * K, sizeof(double));
    double *rhs = (double *)calloc((size_t)K, sizeof(double));
    double *p = (double *)malloc((size_t)K * sizeof(double));
    for (int64_t j = 0; j < m; ++j) {
        for (int k = 0; k < K; ++k) p[k] = fold_p(c, mode, oidx, j, k);
        for (int k1 = 0; k1 < K; ++k1) {
            for (int k2 = 0; k2 < K; ++k2) M[k1 * K + k2] += p[k1] * p[k2];
            rhs[k1] += vals[j] * p[k1];
        }
    }
    double lam = c->reg_mode ? c->lambda * (double)m : c->lambda;
    for (int k = 0; k < K; ++k) M[k * K + k] += lam;
    int rc = cholesky_solve(K, M, rhs, row_out);
    free(M); free(rhs); free(p);
    return rc == 0 ? OR_OK : OR_E_NUMERIC;
}

/* CDTF fold-in of one new row: start from a = 0 (so r = x), then `sweeps`
 * passes over the columns k = 0..K-1, each the C = 1 update of eq. (SALS):
 *   rhat = r + a_k p_k;  a_k = sum rhat p_k / (lambda_i + sum p_k^2);
 *   r = rhat - a_k p_k. */
int or_foldin_cdtf(const or_ctx *c, int mode, int64_t m, const int32_t *oidx,
                   const double *vals, int sweeps, double *row_out)
{
    if (check_fold(c, mode, m, oidx, vals) != OR_OK || sweeps < 1) return OR_E_INVALID;
    int K = c->K;
    for (int k = 0; k < K; ++k) row_out[k] = 0.0;
    if (m == 0) return OR_OK;
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *rh = (double *)malloc((size_t)m * sizeof(double));
    for (int64_t j = 0; j < m; ++j) r[j] = vals[j];
    double lam = c->reg_mode ? c->lambda * (double)m : c->lambda;
    for (int s = 0; s < sweeps; ++s) {
        for (int k = 0; k < K; ++k) {
            double num = 0.0, den = 0.0;
            for (int64_t j = 0; j < m; ++j) {
                double pk = fold_p(c, mode, oidx, j, k);
                rh[j] = r[j] + row_out[k] * pk;
                num += rh[j] * pk;
                den += pk * pk;
            }
            double ak = num / (lam + den);
            row_out[k] = ak;
            for (int64_t j = 0; j < m; ++j) r[j] = rh[j] - ak * fold_p(c, mode, oidx, j, k);
        }
    }
    free(r); free(rh);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Initial factors the library draws by itself (Section 3.1: A^(1) = 0 and
 * the other factors random, so that R = X).  The generator is SplitMix64
 * (Steele, Lea, Flood, OOPSLA 2014) used as a counter-based generator: the
 * t-th output for seed s is mix(s + t * 0x9E3779B97F4A7C15), t = 1, 2, ...
 * Entry (n, i, k) takes counter t = 1 + offset_n + i*K + k with
 * offset_n = K * sum_{l<n} I_l; its value is u / sqrt(K) where u is the top
 * 53 bits of the output scaled to [0, 1). */
uint64_t or_splitmix64(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + t * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Random column order of sweep t (Algorithm 1 picks each split's columns
 * without replacement), the rule the library uses when asked for random
 * orders: start from 0..K-1; walk i from K-1 down to 1; draw the SplitMix64
 * output of counter 2^62 + t*K + i, keep its top 53 bits u, and swap
 * positions i and floor(u * (i + 1) / 2^53), an index in [0, i]
 * (Fisher and Yates' shuffle, in Durstenfeld's in-place form). */
void or_column_order(uint64_t seed, int64_t t, int K, int32_t *out)
{
    for (int k = 0; k < K; ++k) out[k] = k;
    for (int i = K - 1; i > 0; --i) {
        uint64_t counter = ((uint64_t)1 << 62) + (uint64_t)t * (uint64_t)K + (uint64_t)i;
        uint64_t u = or_splitmix64(seed, counter) >> 11;
        unsigned __int128 prod = (unsigned __int128)u * (unsigned __int128)(uint64_t)(i + 1);
        int j = (int)(uint64_t)(prod >> 53);
        int32_t tmp = out[i];
        out[i] = out[j];
        out[j] = tmp;
    }
}

void or_init_factors(or_ctx *c, uint64_t seed, int first_factor_zero)
{
    uint64_t offset = 0;
    double scale = sqrt((double)c->K);
    for (int n = 0; n < c->N; ++n) {
        for (int64_t i = 0; i < c->dims[n]; ++i) {
            for (int k = 0; k < c->K; ++k) {
                double v = 0.0;
                if (!(first_factor_zero && n == 0)) {
                    uint64_t t = 1 + offset + (uint64_t)i * (uint64_t)c->K + (uint64_t)k;
                    double u = (double)(or_splitmix64(seed, t) >> 11) * (1.0 / 9007199254740992.0);
                    v = u / scale;
                }
                c->A[n][i * c->K + k] = v;
            }
        }
        offset += (uint64_t)c->dims[n] * (uint64_t)c->K;
    }
}
