/* Host sanitizer run of the FP64 oracle and the input generators: every
 * oracle entry point on small seeded tensors (uniform and Zipf, repeated
 * tuples, empty rows, C not dividing K, both regularisers, a pivot failure,
 * fold-in of empty and non-empty requests).  Built with
 * -fsanitize=address,undefined by the CPU tests; exits non-zero on any
 * unexpected status, and the sanitizers abort on any memory or UB error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct or_ctx or_ctx;
int or_create(int N, const int64_t *dims, int64_t nnz, const int32_t *idx, const double *vals,
              int K, double lambda, int reg_mode, or_ctx **out);
void or_destroy(or_ctx *c);
void or_set_threads(int t);
int or_set_factor(or_ctx *c, int n, const double *h);
int or_get_factor(const or_ctx *c, int n, double *h);
int or_get_csr(const or_ctx *c, int n, int64_t *rowptr, int32_t *perm);
void or_get_residual(const or_ctx *c, double *h);
void or_resync(or_ctx *c);
int or_split(or_ctx *c, int ncols, const int32_t *cols, int T_in);
int or_sweep(or_ctx *c, int C, int T_in, const int32_t *order);
int or_row_update(const or_ctx *c, int n, int64_t i, int ncols, const int32_t *cols, double *a);
int64_t or_bad_row(const or_ctx *c);
void or_loss(const or_ctx *c, double *loss, double *rmse);
int or_predict(const or_ctx *c, int64_t m, const int32_t *q, double *out);
int or_foldin_full(const or_ctx *c, int mode, int64_t m, const int32_t *oidx, const double *vals,
                   double *row);
int or_foldin_cdtf(const or_ctx *c, int mode, int64_t m, const int32_t *oidx, const double *vals,
                   int sweeps, double *row);
void or_init_factors(or_ctx *c, uint64_t seed, int first_factor_zero);
void or_column_order(uint64_t seed, int64_t t, int K, int32_t *out);

int64_t synth_tuples(uint64_t seed, int N, const int64_t *dims, int64_t ndraw, int dist,
                     double zipf_s, int dedupe, int32_t *out, int64_t cap);
int synth_values(uint64_t seed, int N, const int64_t *dims, int64_t nnz, const int32_t *idx, int R,
                 int scale, double sigma, double *out);
void synth_factor(uint64_t seed, int n, int64_t I, int K, int zero, double *out);
void synth_permutation(uint64_t seed, uint64_t stream, int64_t n, int32_t *out);
void synth_mask(uint64_t seed, uint64_t stream, int64_t n, double p, uint8_t *out);
int synth_zipf_ints(uint64_t seed, uint64_t stream, int64_t count, double s, int64_t hi, int32_t *out);
void synth_uniform_ints(uint64_t seed, uint64_t stream, int64_t count, int64_t n, int32_t *out);
void synth_exponential(uint64_t seed, uint64_t stream, int64_t count, double rate, double *out);
int synth_request_values(uint64_t data_seed, int N, const int64_t *dims, int R, uint64_t req_seed,
                         int64_t nreq, const int64_t *req_ptr, const int32_t *oidx, double sigma,
                         double *out);

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            exit(1);                                                         \
        }                                                                    \
    } while (0)

static void run_case(int N, const int64_t *dims, int64_t ndraw, int dist, int dedupe, int K, int C,
                     int reg, uint64_t seed)
{
    int32_t *idx = malloc((size_t)ndraw * N * sizeof(int32_t));
    int64_t nnz = synth_tuples(seed, N, dims, ndraw, dist, 1.0, dedupe, idx, ndraw);
    CHECK(nnz > 0);
    double *x = malloc((size_t)nnz * sizeof(double));
    CHECK(synth_values(seed, N, dims, nnz, idx, 3, 1, 0.1, x) == 0);
    or_ctx *c = NULL;
    CHECK(or_create(N, dims, nnz, idx, x, K, 0.3, reg, &c) == 0);
    for (int n = 0; n < N; ++n) {
        double *A = malloc((size_t)dims[n] * K * sizeof(double));
        synth_factor(seed + 7, n, dims[n], K, n == 0, A);
        CHECK(or_set_factor(c, n, A) == 0);
        CHECK(or_get_factor(c, n, A) == 0);
        free(A);
        int64_t *rp = malloc((size_t)(dims[n] + 1) * sizeof(int64_t));
        int32_t *pm = malloc((size_t)nnz * sizeof(int32_t));
        CHECK(or_get_csr(c, n, rp, pm) == 0);
        CHECK(rp[dims[n]] == nnz);
        free(rp);
        free(pm);
    }
    or_resync(c);
    int32_t *order = malloc((size_t)K * sizeof(int32_t));
    or_column_order(seed, 0, K, order);
    CHECK(or_sweep(c, C, 2, order) == 0);
    CHECK(or_split(c, 1, order, 1) == 0);
    double a[64];
    CHECK(or_row_update(c, N - 1, dims[N - 1] - 1, C < 64 ? C : 64, order, a) == 0);
    double loss, rmse;
    or_loss(c, &loss, &rmse);
    CHECK(isfinite(loss) && isfinite(rmse));
    double *r = malloc((size_t)nnz * sizeof(double));
    or_get_residual(c, r);
    double *pred = malloc((size_t)nnz * sizeof(double));
    CHECK(or_predict(c, nnz, idx, pred) == 0);
    for (int64_t j = 0; j < nnz; ++j) CHECK(fabs(x[j] - pred[j] - r[j]) < 1e-8);
    /* fold-in: an empty request and one of 40 entries */
    int64_t ptr[3] = {0, 0, 40};
    int32_t *oidx = malloc(40 * (size_t)(N - 1) * sizeof(int32_t));
    for (int t = 0; t < N - 1; ++t) {
        int32_t *col = malloc(40 * sizeof(int32_t));
        synth_uniform_ints(seed, 510 + t, 40, dims[t + 1], col);
        for (int j = 0; j < 40; ++j) oidx[j * (N - 1) + t] = col[j];
        free(col);
    }
    double vals[40];
    CHECK(synth_request_values(seed, N, dims, 3, seed + 1, 2, ptr, oidx, 0.25, vals) == 0);
    double *row = malloc((size_t)K * sizeof(double));
    CHECK(or_foldin_full(c, 0, 0, oidx, vals, row) == 0);
    CHECK(or_foldin_full(c, 0, 40, oidx, vals, row) == 0);
    CHECK(or_foldin_cdtf(c, 0, 40, oidx, vals, 3, row) == 0);
    or_init_factors(c, seed, 1);
    or_destroy(c);
    free(idx); free(x); free(order); free(r); free(pred); free(oidx); free(row);
}

int main(void)
{
    or_set_threads(2);
    const int64_t d3[3] = {30, 20, 25}, d4[4] = {12, 9, 7, 5}, d2[2] = {40, 1};
    run_case(3, d3, 2000, 0, 2, 7, 3, 0, 11);     /* uniform, distinct, C does not divide K */
    run_case(4, d4, 1500, 1, 1, 5, 5, 1, 12);     /* Zipf, repeats dropped, C = K, weighted */
    run_case(3, d3, 800, 1, 0, 6, 1, 0, 13);      /* multiset, CDTF, empty rows */
    run_case(2, d2, 30, 0, 0, 2, 2, 0, 14);       /* one-row mode */

    /* a non-positive pivot: a factor row of 1e200 makes B infinite */
    {
        const int64_t d[3] = {6, 5, 4};
        int32_t idx[60 * 3];
        int64_t nnz = synth_tuples(21, 3, d, 60, 0, 1.0, 2, idx, 60);
        double x[60];
        CHECK(synth_values(21, 3, d, nnz, idx, 2, 0, 0.1, x) == 0);
        or_ctx *c = NULL;
        CHECK(or_create(3, d, nnz, idx, x, 3, 0.1, 0, &c) == 0);
        double A[6 * 3];
        for (int n = 1; n < 3; ++n) {
            synth_factor(22, n, d[n], 3, 0, A);
            if (n == 1) for (int k = 0; k < 3; ++k) A[2 * 3 + k] = 1e200;
            or_set_factor(c, n, A);
        }
        int32_t order[3] = {0, 1, 2};
        CHECK(or_sweep(c, 3, 1, order) == 4);
        CHECK(or_bad_row(c) >= 0);
        or_destroy(c);
    }

    /* generators on their own */
    int32_t perm[100];
    synth_permutation(3, 4, 100, perm);
    uint8_t mask[100];
    synth_mask(3, 5, 100, 0.1, mask);
    int32_t z[200];
    CHECK(synth_zipf_ints(3, 6, 200, 1.1, 5000, z) == 0);
    double e[50];
    synth_exponential(3, 7, 50, 1000.0, e);
    /* invalid inputs are refused */
    {
        int32_t bad[2] = {5, 0};
        const int64_t d[2] = {2, 2};
        double v = 1.0;
        or_ctx *c = NULL;
        CHECK(or_create(2, d, 1, bad, &v, 1, 1.0, 0, &c) != 0 && c == NULL);
    }
    printf("sanitized oracle and generators ok\n");
    return 0;
}
