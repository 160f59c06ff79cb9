/*
 * synth.c -- seeded synthetic inputs for the SALS / CDTF tests and benchmark.
 *
 * This module only draws inputs: index tuples, observed values from a random
 * low-rank ground truth plus Gaussian noise, starting factors, column orders,
 * held-out masks and fold-in request streams.  It holds none of the method's
 * arithmetic and is shared, as input, by the oracle runs and the GPU runs.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a
 * counter-based generator.  Output t (t = 0, 1, ...) of stream s under seed
 * `seed` is mix(key(seed, s) + (t + 1) * 0x9E3779B97F4A7C15) with
 * key(seed, s) = mix(seed ^ (s * 0xD1B54A32D192ED03)), so every value depends
 * only on (seed, stream, counter) and the multi-threaded loops give the same
 * result for any thread count.
 *
 * Distributions:
 *   uniform integer in [0, n):  high 64 bits of the 128-bit product out * n
 *   uniform double in [0, 1):   (out >> 11) * 2^-53
 *   normal:                     Box-Muller, cos branch, from counters 2t, 2t+1
 *   Zipf(s) on ranks 1..n:      Walker/Vose alias table over p(r) ~ r^-s
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t skey(uint64_t seed, uint64_t stream)
{
    return mix64(seed ^ (stream * 0xD1B54A32D192ED03ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t t) { return mix64(key + (t + 1) * GAMMA); }

static inline double u01(uint64_t v) { return (double)(v >> 11) * (1.0 / 9007199254740992.0); }

static inline uint64_t below(uint64_t v, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)v * (unsigned __int128)n) >> 64);
}

static inline double normal01(uint64_t key, uint64_t t)
{
    double u1 = 1.0 - u01(draw(key, 2 * t));      /* (0, 1] */
    double u2 = u01(draw(key, 2 * t + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

uint64_t synth_draw(uint64_t seed, uint64_t stream, uint64_t t) { return draw(skey(seed, stream), t); }

/* ---------------------------------------------------------------------- */
/* Alias table (Vose) for p(r) ~ (r+1)^-s, r = 0..n-1. */
typedef struct { double *prob; int64_t *alias; int64_t n; } alias_t;

static int alias_build(alias_t *a, int64_t n, double s)
{
    a->n = n;
    a->prob = (double *)malloc((size_t)n * sizeof(double));
    a->alias = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    int64_t *small = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *large = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!a->prob || !a->alias || !w || !small || !large) return -1;
    double tot = 0.0;
    for (int64_t r = 0; r < n; ++r) { w[r] = pow((double)(r + 1), -s); tot += w[r]; }
    int64_t ns = 0, nl = 0;
    for (int64_t r = 0; r < n; ++r) {
        w[r] = w[r] * (double)n / tot;
        if (w[r] < 1.0) small[ns++] = r; else large[nl++] = r;
    }
    while (ns > 0 && nl > 0) {
        int64_t l = small[--ns], g = large[--nl];
        a->prob[l] = w[l];
        a->alias[l] = g;
        w[g] = (w[g] + w[l]) - 1.0;
        if (w[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { int64_t g = large[--nl]; a->prob[g] = 1.0; a->alias[g] = g; }
    while (ns > 0) { int64_t l = small[--ns]; a->prob[l] = 1.0; a->alias[l] = l; }
    free(w); free(small); free(large);
    return 0;
}

static void alias_free(alias_t *a) { free(a->prob); free(a->alias); }

static inline int64_t alias_draw(const alias_t *a, uint64_t v1, uint64_t v2)
{
    int64_t r = (int64_t)below(v1, (uint64_t)a->n);
    return u01(v2) < a->prob[r] ? r : a->alias[r];
}

/* Fisher-Yates permutation of 0..n-1 from stream `stream`. */
void synth_permutation(uint64_t seed, uint64_t stream, int64_t n, int32_t *out)
{
    uint64_t key = skey(seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)i;
    for (int64_t i = n - 1; i >= 1; --i) {
        int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = out[i]; out[i] = out[j]; out[j] = t;
    }
}

/* ---------------------------------------------------------------------- */
/* Stable LSD radix sort of (key, payload) pairs, 8-bit digits. */
static void radix_sort_pairs(uint64_t *k, uint64_t *v, int64_t n, uint64_t *tk, uint64_t *tv)
{
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)calloc((size_t)nt * 256, sizeof(int64_t));
    for (int pass = 0; pass < 8; ++pass) {
        int sh = pass * 8;
        memset(hist, 0, (size_t)nt * 256 * sizeof(int64_t));
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t *h = hist + (int64_t)t * 256;
            for (int64_t i = lo; i < hi; ++i) h[(k[i] >> sh) & 255] += 1;
        }
        /* skip a pass whose digit is the same for every key */
        int nonzero = 0;
        for (int d = 0; d < 256; ++d) {
            int64_t s = 0;
            for (int t = 0; t < nt; ++t) s += hist[t * 256 + d];
            if (s) nonzero += 1;
        }
        if (nonzero <= 1) continue;
        int64_t run = 0;
        for (int d = 0; d < 256; ++d)
            for (int t = 0; t < nt; ++t) {
                int64_t c = hist[t * 256 + d];
                hist[t * 256 + d] = run;
                run += c;
            }
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t *h = hist + (int64_t)t * 256;
            for (int64_t i = lo; i < hi; ++i) {
                int64_t p = h[(k[i] >> sh) & 255]++;
                tk[p] = k[i];
                tv[p] = v[i];
            }
        }
        memcpy(k, tk, (size_t)n * sizeof(uint64_t));
        memcpy(v, tv, (size_t)n * sizeof(uint64_t));
    }
    free(hist);
}

/* Draw one index tuple (counter t) into out[0..N). */
static void draw_tuple(int N, const int64_t *dims, const uint64_t *keys, const alias_t *zipf,
                       const int32_t *const *rank2idx, uint64_t t, int32_t *out)
{
    for (int n = 0; n < N; ++n) {
        if (zipf) {
            int64_t r = alias_draw(&zipf[n], draw(keys[n], 2 * t), draw(keys[n], 2 * t + 1));
            out[n] = rank2idx[n][r];
        } else {
            out[n] = (int32_t)below(draw(keys[n], t), (uint64_t)dims[n]);
        }
    }
}

static uint64_t tuple_key(int N, const int64_t *dims, const int32_t *tu, int exact)
{
    if (exact) {
        uint64_t k = 0;
        for (int n = 0; n < N; ++n) k = k * (uint64_t)dims[n] + (uint64_t)tu[n];
        return k;
    }
    uint64_t h = 0x243F6A8885A308D3ULL;
    for (int n = 0; n < N; ++n) h = mix64(h ^ ((uint64_t)(uint32_t)tu[n] + (uint64_t)n * GAMMA));
    return h;
}

/*
 * Index tuples, nnz x N row-major into out (capacity `cap` tuples).
 *   dist   0: every mode uniform on [0, dims[n]);
 *          1: every mode Zipf(zipf_s) over ranks, rank mapped to an index by a
 *             seeded permutation per mode.
 *   dedupe 0: keep all `ndraw` draws (a multiset);
 *          1: drop repeats, keeping the first draw of each tuple;
 *          2: exactly `ndraw` distinct tuples: repeats are dropped and more
 *             draws are taken until the count is reached (rejection).
 * Returns the number of tuples written, or -1 on failure.
 */
int64_t synth_tuples(uint64_t seed, int N, const int64_t *dims, int64_t ndraw, int dist,
                     double zipf_s, int dedupe, int32_t *out, int64_t cap)
{
    uint64_t keys[8];
    alias_t zipf[8];
    int32_t *r2i[8] = {0};
    for (int n = 0; n < N; ++n) keys[n] = skey(seed, 10 + (uint64_t)n);
    if (dist == 1) {
        for (int n = 0; n < N; ++n) {
            if (alias_build(&zipf[n], dims[n], zipf_s) != 0) return -1;
            r2i[n] = (int32_t *)malloc((size_t)dims[n] * sizeof(int32_t));
            synth_permutation(seed, 30 + (uint64_t)n, dims[n], r2i[n]);
        }
    }
    const alias_t *zp = dist == 1 ? zipf : NULL;
    double space = 1.0;
    for (int n = 0; n < N; ++n) space *= (double)dims[n];
    int exact = space < 9.0e18;
    if (dedupe == 2 && space < (double)ndraw) return -1;

    int64_t want = ndraw;
    if (want > cap) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < want; ++t)
        draw_tuple(N, dims, keys, zp, (const int32_t *const *)r2i, (uint64_t)t, out + t * N);
    int64_t count = want;
    uint64_t next_t = (uint64_t)want;

    if (dedupe != 0) {
        for (;;) {
            uint64_t *k = (uint64_t *)malloc((size_t)count * sizeof(uint64_t));
            uint64_t *v = (uint64_t *)malloc((size_t)count * sizeof(uint64_t));
            uint64_t *tk = (uint64_t *)malloc((size_t)count * sizeof(uint64_t));
            uint64_t *tv = (uint64_t *)malloc((size_t)count * sizeof(uint64_t));
            uint8_t *keep = (uint8_t *)malloc((size_t)count);
            if (!k || !v || !tk || !tv || !keep) return -1;
#pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < count; ++t) {
                k[t] = tuple_key(N, dims, out + t * N, exact);
                v[t] = (uint64_t)t;
                keep[t] = 1;
            }
            radix_sort_pairs(k, v, count, tk, tv);
            free(tk); free(tv);
            /* within a run of equal keys the payloads ascend (stable sort):
             * the first is the earliest draw; later equal tuples are dropped */
            int64_t dropped = 0;
            for (int64_t s = 0; s < count;) {
                int64_t e = s + 1;
                while (e < count && k[e] == k[s]) ++e;
                for (int64_t q = s + 1; q < e; ++q) {
                    const int32_t *tq = out + (int64_t)v[q] * N;
                    for (int64_t p = s; p < q; ++p) {
                        if (!keep[v[p]]) continue;
                        if (memcmp(tq, out + (int64_t)v[p] * N, (size_t)N * sizeof(int32_t)) == 0) {
                            keep[v[q]] = 0;
                            dropped += 1;
                            break;
                        }
                    }
                }
                s = e;
            }
            free(k); free(v);
            if (dropped) {
                int64_t w = 0;
                for (int64_t t = 0; t < count; ++t) {
                    if (!keep[t]) continue;
                    if (w != t) memmove(out + w * N, out + t * N, (size_t)N * sizeof(int32_t));
                    w += 1;
                }
                count = w;
            }
            free(keep);
            if (dedupe == 1 || count == want || dropped == 0) break;
            /* rejection: draw the missing tuples from fresh counters */
            int64_t miss = want - count;
            for (int64_t q = 0; q < miss; ++q)
                draw_tuple(N, dims, keys, zp, (const int32_t *const *)r2i, next_t + (uint64_t)q,
                           out + (count + q) * N);
            next_t += (uint64_t)miss;
            count = want;
        }
    }
    if (dist == 1)
        for (int n = 0; n < N; ++n) { alias_free(&zipf[n]); free(r2i[n]); }
    return count;
}

/* Ground-truth factor G^(n) (dims[n] x R, entries U(0,1)) of stream 100+n. */
static double *truth_factor(uint64_t seed, int n, int64_t I, int R)
{
    double *G = (double *)malloc((size_t)I * (size_t)R * sizeof(double));
    if (!G) return NULL;
    uint64_t key = skey(seed, 100 + (uint64_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < I * R; ++t) G[t] = u01(draw(key, (uint64_t)t));
    return G;
}

/*
 * Observed values x_j = f(v_j) + sigma * z_j with v_j = sum_{k<R} prod_n
 * G^(n)[i_n, k] (ground truth of rank R) and z_j standard normal (stream 200).
 *   scale 0: f(v) = v;  scale 1: f(v) = 1 + 4 v / R  (maps [0, R] to [1, 5]).
 */
int synth_values(uint64_t seed, int N, const int64_t *dims, int64_t nnz, const int32_t *idx,
                 int R, int scale, double sigma, double *out)
{
    double *G[8];
    for (int n = 0; n < N; ++n) {
        G[n] = truth_factor(seed, n, dims[n], R);
        if (!G[n]) return -1;
    }
    uint64_t nkey = skey(seed, 200);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nnz; ++j) {
        double v = 0.0;
        for (int k = 0; k < R; ++k) {
            double p = 1.0;
            for (int n = 0; n < N; ++n) p *= G[n][(int64_t)idx[j * N + n] * R + k];
            v += p;
        }
        double f = scale ? 1.0 + 4.0 * v / (double)R : v;
        out[j] = f + sigma * normal01(nkey, (uint64_t)j);
    }
    for (int n = 0; n < N; ++n) free(G[n]);
    return 0;
}

/* Starting factors: U(0,1)/sqrt(K) (stream 300+n); factor 0 zero when asked. */
void synth_factor(uint64_t seed, int n, int64_t I, int K, int zero, double *out)
{
    uint64_t key = skey(seed, 300 + (uint64_t)n);
    double s = sqrt((double)K);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < I * (int64_t)K; ++t)
        out[t] = zero ? 0.0 : u01(draw(key, (uint64_t)t)) / s;
}

/* mask[j] = 1 with probability p (stream `stream`). */
void synth_mask(uint64_t seed, uint64_t stream, int64_t n, double p, uint8_t *out)
{
    uint64_t key = skey(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) out[j] = u01(draw(key, (uint64_t)j)) < p ? 1 : 0;
}

/* Zipf(s) integers on [1, hi] (request sizes). */
int synth_zipf_ints(uint64_t seed, uint64_t stream, int64_t count, double s, int64_t hi,
                    int32_t *out)
{
    alias_t a;
    if (alias_build(&a, hi, s) != 0) return -1;
    uint64_t key = skey(seed, stream);
    for (int64_t t = 0; t < count; ++t)
        out[t] = (int32_t)(alias_draw(&a, draw(key, 2 * (uint64_t)t), draw(key, 2 * (uint64_t)t + 1)) + 1);
    alias_free(&a);
    return 0;
}

/* Uniform integers on [0, n). */
void synth_uniform_ints(uint64_t seed, uint64_t stream, int64_t count, int64_t n, int32_t *out)
{
    uint64_t key = skey(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) out[t] = (int32_t)below(draw(key, (uint64_t)t), (uint64_t)n);
}

/* Exponential gaps with the given rate (Poisson arrivals). */
void synth_exponential(uint64_t seed, uint64_t stream, int64_t count, double rate, double *out)
{
    uint64_t key = skey(seed, stream);
    for (int64_t t = 0; t < count; ++t) out[t] = -log(1.0 - u01(draw(key, (uint64_t)t))) / rate;
}

/*
 * Fold-in request values: new rows of mode 0.  Request q has a ground-truth
 * row g_q ~ U(0,1)^R (stream 400, counter q*R + k); an entry with other-mode
 * indices (i_2..i_N) gets x = 1 + 4 (sum_k g_qk prod_{l>=2} G^(l)[i_l,k]) / R
 * + sigma z, with G^(l) the training data's ground truth (same data seed) and
 * z from stream 401 under the request seed.
 */
int synth_request_values(uint64_t data_seed, int N, const int64_t *dims, int R, uint64_t req_seed,
                         int64_t nreq, const int64_t *req_ptr, const int32_t *oidx, double sigma,
                         double *out)
{
    double *G[8] = {0};
    for (int n = 1; n < N; ++n) {
        G[n] = truth_factor(data_seed, n, dims[n], R);
        if (!G[n]) return -1;
    }
    uint64_t gkey = skey(req_seed, 400), nkey = skey(req_seed, 401);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nreq; ++q) {
        for (int64_t j = req_ptr[q]; j < req_ptr[q + 1]; ++j) {
            double v = 0.0;
            for (int k = 0; k < R; ++k) {
                double p = u01(draw(gkey, (uint64_t)q * (uint64_t)R + (uint64_t)k));
                for (int n = 1; n < N; ++n) p *= G[n][(int64_t)oidx[j * (N - 1) + (n - 1)] * R + k];
                v += p;
            }
            out[j] = 1.0 + 4.0 * v / (double)R + sigma * normal01(nkey, (uint64_t)j);
        }
    }
    for (int n = 1; n < N; ++n) free(G[n]);
    return 0;
}

void synth_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
