/*
 * tf.h -- C ABI of the MI355X SALS / CDTF sparse tensor-factorisation path.
 *
 * Problem (Definition 1, eq. (TF) of Shin & Kang, arXiv:1410.5209): given the
 * observed entries Omega of an N-way tensor X, a rank K and lambda > 0, find
 * factor matrices A^(n) (I_n x K) minimising
 *     sum_{Omega} (x - sum_k prod_n a^(n)_{i_n k})^2 + lambda sum_n ||A^(n)||_F^2.
 * The library runs Algorithm 1 (serial SALS) on one GPU: one outer iteration
 * walks the K columns in blocks of C, updating every row of every factor by
 * eq. (SALS) and keeping the residual tensor R of eq. (SALS_R) up to date.
 * C = 1 is CDTF; C = K with one inner iteration is ALS (eq. (ALS)).
 *
 * Conventions for every call:
 *  - Every call returns tf_status (TF_OK = 0); no exception crosses the ABI.
 *    tf_last_error() returns a message for the last failure on that context.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary host memory.  The caller keeps ownership of every
 *    buffer it passes; the library copies what it needs and never frees them.
 *  - Work runs on the stream given in tf_options (NULL = the null stream).
 *    Calls that return values to the host synchronise that stream.
 *  - A context is used by one host thread at a time, except the tf_serve_*
 *    calls, which are thread-safe.
 *  - Indices are 0-based int32; index tuples are row-major (entry j occupies
 *    idx[j*N .. j*N+N-1]); factors are row-major I_n x K.
 */
#ifndef TF_SALS_H
#define TF_SALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tf_status;
#define TF_OK 0
#define TF_E_INVALID 1      /* an argument breaks a documented rule */
#define TF_E_NOMEM 2        /* device or host allocation failed */
#define TF_E_DEVICE 3       /* a HIP runtime call failed, or no GPU */
#define TF_E_NUMERIC 4      /* a Cholesky pivot was not positive */
#define TF_E_UNSUPPORTED 5  /* a valid request this build does not run */
#define TF_E_BUSY 6         /* serving queue full */
#define TF_E_STATE 7        /* call not allowed in the context's state */

/* Arithmetic of the path. In every mode the C x C Cholesky solve and the
 * loss reduction run in FP64. */
#define TF_PREC_F64 0   /* factors, residual, Gram accumulation: FP64 */
#define TF_PREC_F32 1   /* factors, residual, Gram accumulation: FP32 */
#define TF_PREC_BF16 2  /* factors BF16 (round to nearest even); residual and
                           Gram accumulation FP32 */

/* How rows are mapped to the GPU in a mode pass. */
#define TF_STRATEGY_PLAIN 0  /* one wavefront per non-empty row, in row order */
#define TF_STRATEGY_SKEW 1   /* rows bucketed by length (1..64 lanes per row),
                                rows above split_threshold cut into chunks whose
                                partial Gram matrices are summed in a fixed order */
#define TF_STRATEGY_AUTO 2   /* SKEW, with each mode's row tiles chosen by timed
                                trial passes (as tf_autotune with the one
                                candidate C, tune_tiles = 1) before the first
                                split of each new compute width */
#define TF_STRATEGY_PERSISTENT 3  /* SKEW's plan in one persistent launch per
                                pass: as many workgroups as the GPU holds at
                                once, whose wavefronts take the tasks (chunks
                                of the longest rows first, then groups of
                                shorter rows) from a counter until none is
                                left; same results as SKEW, bit for bit */

/* Column order of tf_sweep (Algorithm 1 draws each split's columns without
 * replacement; Section 3.1 keeps a fixed order for CDTF). */
#define TF_ORDER_FIXED 0     /* the order set by tf_set_col_order (initially
                                0..K-1): blocks of C consecutive entries */
#define TF_ORDER_RANDOM 1    /* every tf_sweep first draws a permutation:
                                sweep t (0, 1, ... counted per context) runs
                                Fisher-Yates, for i = K-1 down to 1 swapping
                                entries i and j = floor(u (i+1) / 2^53), where
                                u is the top 53 bits of SplitMix64 output
                                2^62 + t K + i for the context's seed (the
                                generator the factor initialisation uses);
                                tf_get_col_order returns it */

/* Device memory hooks: alloc returns `bytes` of device memory on the
 * context's device, aligned to 256 bytes, or NULL; free releases a block
 * alloc returned (bytes is the size it was asked for).  stream is the
 * context's stream.  Both may be called from a serving thread. */
typedef void *(*tf_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*tf_free_fn)(void *ptr, size_t bytes, void *stream, void *user);

typedef struct tf_options {
    uint32_t size;             /* sizeof(tf_options): versions the struct */
    int32_t precision;         /* TF_PREC_* (default TF_PREC_F32) */
    int32_t reg_mode;          /* 0: lambda as in eq. (TF) (default);
                                  1: weighted lambda, row i of mode n uses
                                     lambda * |Omega^(n)_i| (Section 5.1.3) */
    int32_t first_factor_zero; /* 1 (default): A^(1) = 0 so that R = X
                                  (Section 3.1); 0: all factors random */
    int32_t strategy;          /* TF_STRATEGY_* (default TF_STRATEGY_SKEW) */
    uint64_t seed;             /* seed of the factor initialisation and of
                                  TF_ORDER_RANDOM (default 2) */
    void *stream;              /* hipStream_t, NULL = null stream */
    int32_t lane_nnz;          /* SKEW: target nonzeros per lane (0 = 2) */
    int32_t split_threshold;   /* SKEW: rows longer than this are split
                                  (0 = 4096) */
    int32_t chunk_nnz;         /* SKEW: nonzeros per chunk of a split row
                                  (0 = 2048) */
    int32_t resid_share;       /* TF_RESID_*: where the row passes of modes
                                  2..N read R-hat (default TF_RESID_AUTO) */
    int32_t col_order;         /* TF_ORDER_* (default TF_ORDER_FIXED) */
    size_t mem_budget;         /* device bytes the context may hold at once,
                                  serving slots and call workspaces included;
                                  an allocation beyond it fails with
                                  TF_E_NOMEM (0 = no limit) */
    tf_alloc_fn dev_alloc;     /* NULL (default): hipMalloc / hipFree; else */
    tf_free_fn dev_free;       /*   every device allocation of the context */
    void *alloc_user;          /*   goes through these two (both set) */
    int32_t graph;             /* 1: a tf_sweep whose starting state (C, T_in,
                                  pending columns, residual placement, row
                                  plans, buffers) repeats the previous sweep's
                                  is captured as one HIP graph, and later
                                  sweeps with that state replay it (one launch
                                  instead of one per kernel: for tensors small
                                  enough to be launch-bound).  0 (default):
                                  every sweep launches its kernels.  Results
                                  do not depend on it.  A sweep that cannot be
                                  captured runs without a graph, and
                                  tf_last_error then says why. */
} tf_options;

/* Residual placement.  Mode 1 keeps R-hat in its own row order and forms it
 * in its first pass of each split (eq. (SALS_R) of the previous split plus
 * the R-hat step of Algorithm 1), which needs the previous split's final and
 * this split's starting columns of every factor row it gathers.  Another
 * mode either keeps its own copy the same way (TF_RESID_OWN) or reads mode
 * 1's copy through a permutation (TF_RESID_SHARED: one random 4- or 8-byte
 * read per entry and pass, no residual work).  TF_RESID_AUTO picks, per
 * mode and split, the choice with fewer random cache-line requests per
 * entry given the split's slab layout and T_in.  The choice changes only
 * rounding. */
#define TF_RESID_AUTO 0
#define TF_RESID_OWN 1
#define TF_RESID_SHARED 2

typedef struct tf_ctx tf_ctx;

/* Fill *opt with the defaults above (size set). */
void tf_default_options(tf_options *opt);

/*
 * tf_init -- build the model state from the observed entries.
 *   N       modes, 2 <= N <= 8
 *   dims    host[N], 1 <= I_n <= 2^31 - 1
 *   nnz     number of observed entries, 1 <= nnz <= 2^31 - 1
 *   d_idx   device, nnz x N int32 index tuples (row-major); the input order
 *           defines the entry id j used by tf_get_residual and tf_get_csr.
 *           A repeated tuple is one more loss term.
 *   d_vals  device, nnz FP64 observed values
 *   K       rank >= 1;  lambda > 0 (eq. (TF))
 *   opt     NULL for defaults
 * Builds, per mode, the CSR of the row sets Omega^(n)_i (Table 1) with a
 * stable sort (entries keep their input order inside a row), the per-mode
 * copies of the residual, and the row work plan; initialises the factors
 * (SplitMix64 counters, U(0,1)/sqrt(K), A^(1) = 0 unless first_factor_zero
 * is 0) and the residual r = x - reconstruction.  Synchronises the stream.
 * Errors: TF_E_INVALID for a rule above, an index outside [0, I_n) or a
 * non-finite value (the message names the first bad entry); TF_E_NOMEM;
 * TF_E_DEVICE.  On error *out is NULL.
 */
tf_status tf_init(tf_ctx **out, int32_t N, const int64_t *dims, int64_t nnz,
                  const int32_t *d_idx, const double *d_vals, int32_t K, double lambda,
                  const tf_options *opt);

/* Release everything the context owns.  NULL is a no-op. */
void tf_destroy(tf_ctx *ctx);

/* Message of the last failed call on ctx (owned by ctx; "" if none). */
const char *tf_last_error(const tf_ctx *ctx);

/*
 * tf_sweep -- one outer iteration of Algorithm 1.  The current column order
 * (tf_set_col_order; identity by default) is walked in ceil(K/C) blocks of C
 * columns, the last block shorter when C does not divide K.  For each block:
 * R-hat is formed, T_in inner iterations update every row of every mode by
 * eq. (SALS) (FP64 Cholesky, text after Theorem 1), and R is brought up to
 * date by eq. (SALS_R).  1 <= C <= K with C <= 16 (FP64) or C <= 16 or
 * 17..32 (FP32/BF16; run as 32 columns with zero padding); C = 0 uses the
 * width chosen by tf_autotune.  T_in >= 1.  Blocks until done.
 * TF_E_NUMERIC: a pivot was not positive; the message names the mode and
 * the smallest such row of the first mode pass that met one.  The other rows
 * of that pass are updated, those rows keep their previous values, and no
 * factor changes after that pass (the rest of the split and the later splits
 * only keep R consistent), so the state equals that of Algorithm 1 stopped
 * after the failing pass.
 * TF_E_STATE: factors were set without tf_resync.
 */
tf_status tf_sweep(tf_ctx *ctx, int32_t C, int32_t T_in);

/*
 * tf_split -- one block (split) of Algorithm 1 on the given columns:
 * h_cols host[ncols], distinct, in [0, K), with the same width limits as
 * tf_sweep.  Same semantics and errors as one block of tf_sweep.
 */
tf_status tf_split(tf_ctx *ctx, int32_t ncols, const int32_t *h_cols, int32_t T_in);

/* Column order used by tf_sweep: h_order host[K], a permutation of 0..K-1
 * (Algorithm 1 picks columns without replacement; a fixed order is the
 * paper's choice for CDTF, Section 3.1). */
tf_status tf_set_col_order(tf_ctx *ctx, const int32_t *h_order);
tf_status tf_get_col_order(const tf_ctx *ctx, int32_t *h_order);

/*
 * tf_loss -- eq. (TF) in FP64: sum of squared residuals plus lambda times
 * the squared factor norms (weighted by row counts in reg_mode 1).
 * *train_rmse = sqrt(sum r^2 / nnz).  Either output may be NULL.
 */
tf_status tf_loss(tf_ctx *ctx, double *loss, double *train_rmse);

/*
 * tf_predict -- x-hat = sum_k prod_n a^(n)_{i_n k} (the model of eq. (TF))
 * for m query tuples.  d_idx device m x N int32; d_out device m FP64.
 * TF_E_INVALID for an index out of range (nothing written).  m = 0 is a no-op.
 */
tf_status tf_predict(tf_ctx *ctx, int64_t m, const int32_t *d_idx, double *d_out);

/* Factor n as FP64 (host[I_n x K]); set marks the residual stale until
 * tf_resync.  Values are rounded to the storage precision. */
tf_status tf_get_factor(tf_ctx *ctx, int32_t n, double *h);
/* A block of factor n as FP64, host[nrows x ncols] row-major:
 * h[r * ncols + c] = a^(n)_{h_rows[r], h_cols[c]}.  h_rows NULL means all rows
 * in order (nrows must be I_n), h_cols NULL all columns (ncols must be K);
 * entries may repeat.  Reads a few rows or columns of a wide factor without
 * copying all of it.  TF_E_INVALID for a count or an index out of range. */
tf_status tf_get_factor_block(tf_ctx *ctx, int32_t n, int64_t nrows, const int32_t *h_rows,
                              int32_t ncols, const int32_t *h_cols, double *h);
tf_status tf_set_factor(tf_ctx *ctx, int32_t n, const double *h);

/* r = x - reconstruction recomputed from the current factors (definition
 * of R, Section 3.1). */
tf_status tf_resync(tf_ctx *ctx);

/* The maintained residual r, host[nnz] FP64, in input order. */
tf_status tf_get_residual(tf_ctx *ctx, double *h);

/* Mode-n CSR: h_rowptr host[I_n + 1], h_perm host[nnz] (entry ids). */
tf_status tf_get_csr(tf_ctx *ctx, int32_t n, int64_t *h_rowptr, int32_t *h_perm);

/* ------------------------------------------------------------------ */
/* Autotuning of the split width C and of the row tiles per mode.
 * For each candidate C, times one trial split on the GPU: per mode a fused
 * first pass (against a scratch copy of the residual) and, when T_in > 1, a
 * plain pass; the estimated sweep time is ceil(K/C) times that plus slab
 * packing.  Writes only scratch buffers: the model is unchanged.  With
 * tune_tiles, then re-plans each mode over lanes-per-row targets {1,2,4,8}
 * and chunk lengths {1024,4096,16384} (split threshold twice the chunk) for
 * the chosen C and keeps the fastest plan; under TF_STRATEGY_SKEW and
 * TF_STRATEGY_AUTO it then times that plan with both launch forms (one
 * wavefront per task, or one resident grid taking tasks from a counter) and
 * keeps the faster for the mode.  Afterwards tf_sweep(ctx, 0, T_in)
 * uses the chosen C.  Candidates must satisfy 1 <= C <= K and be runnable in
 * the context's precision (C <= 16 in FP64, C <= 16 or C = 32 otherwise;
 * C in 17..31 runs as 32 with zero padding). */
typedef struct tf_tune_result {
    int32_t best_C;
    int32_t ncand;
    int32_t cand_C[16];
    double est_sweep_ms[16];
    int32_t lane_nnz[8], split_threshold[8], chunk_nnz[8];   /* plan per mode */
    double tune_ms;                                          /* wall time of the tuning */
    int32_t persistent[8];   /* launch form per mode: 1 = one resident grid taking
                                tasks from a counter, 0 = one wavefront per task
                                (chosen with the tiles under TF_STRATEGY_SKEW or
                                TF_STRATEGY_AUTO; results do not depend on it) */
} tf_tune_result;
tf_status tf_autotune(tf_ctx *ctx, int32_t T_in, const int32_t *h_cands, int32_t ncand,
                      int32_t tune_tiles, tf_tune_result *out);

/* ------------------------------------------------------------------ */
/* Fold-in: new rows of one mode solved against the resident factors without
 * changing the model (a use of the row update the paper does not make).  A
 * request is the row's observed entries: for each, the indices of the other
 * modes (ascending mode order) and the value.
 *   TF_FOLDIN_FULL: eq. (ALS) for the row, a = (B + lambda_i I_K)^-1 c with c
 *                   built from the values; FP32 (FP64 in FP64 mode) Gram,
 *                   FP64 Cholesky; K <= 128.
 *   TF_FOLDIN_CDTF: `sweeps` passes of the C = 1 update over k = 0..K-1
 *                   starting from a = 0 (CDTF, Section 3.1); FP64 sums.
 * lambda_i = lambda, or lambda * m in reg_mode 1.  An empty request gives 0. */
#define TF_FOLDIN_FULL 0
#define TF_FOLDIN_CDTF 1

/*
 * tf_foldin -- a batch of fold-in requests, synchronously.
 *   mode      0 <= mode < N
 *   nreq      >= 0; h_req_ptr host[nreq + 1] entry offsets (non-decreasing,
 *             h_req_ptr[0] = 0)
 *   d_idx     device, total x (N - 1) int32, total = h_req_ptr[nreq]
 *   d_vals    device, total FP64
 *   d_rows    device, nreq x K FP64 output
 * Every request is solved by its own workgroup, so its result does not
 * depend on the rest of the batch.  TF_E_INVALID for a bad index or value
 * (message names the entry); TF_E_NUMERIC for a non-positive pivot (that
 * row is 0); TF_E_UNSUPPORTED for TF_FOLDIN_FULL with K > 128.
 */
tf_status tf_foldin(tf_ctx *ctx, int32_t mode, int32_t nreq, const int64_t *h_req_ptr,
                    const int32_t *d_idx, const double *d_vals, int32_t method, int32_t sweeps,
                    double *d_rows);

/*
 * tf_foldin_noalloc -- tf_foldin for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, semantics, results (bit for bit) and errors,
 * but the call allocates nothing (no device memory; no host memory either,
 * error messages included).  Its
 * workspace (the products P, chunk tables and partial Gram records, failure
 * flags) lives in one fixed array of 32 MiB per GPU, which the library
 * reserves when it is loaded and holds until the process ends.
 * TF_E_INVALID (message names the bytes needed) for a batch whose workspace
 * exceeds it: about 32 MiB / (K * 4 + 300) entries in FP32, e.g. ~80,000
 * entries at K = 100.  Every call on one GPU uses the same array and it
 * keeps the last call's contents: calls that overlap on one GPU (two host
 * threads, or two streams) race, so the caller serialises them.
 */
tf_status tf_foldin_noalloc(tf_ctx *ctx, int32_t mode, int32_t nreq, const int64_t *h_req_ptr,
                            const int32_t *d_idx, const double *d_vals, int32_t method,
                            int32_t sweeps, double *d_rows);

/* ------------------------------------------------------------------ */
/* Fold-in serving: requests arrive one at a time from any host thread; a
 * scheduler packs whatever is queued into a batch when a stream slot is free
 * and the batch's device bytes fit that slot's share of the memory budget
 * (continuous batching), so batches overlap on the GPU across streams.
 * The resident factors must not change while a server is open. */
typedef struct tf_serve_opts {
    uint32_t size;         /* sizeof(tf_serve_opts) */
    int32_t mode;          /* mode of the new rows (default 0) */
    int32_t method;        /* TF_FOLDIN_* (default TF_FOLDIN_FULL) */
    int32_t sweeps;        /* CDTF sweeps (default 3) */
    int32_t streams;       /* stream slots, >= 1 (default 2) */
    int32_t max_batch;     /* requests per batch (default 512) */
    int32_t queue_cap;     /* queued requests before TF_E_BUSY (default 65536) */
    int64_t mem_budget;    /* device bytes for in-flight batches (default 1 GiB),
                              split evenly over the stream slots */
} tf_serve_opts;

typedef struct tf_request {
    int32_t m;             /* entries */
    const int32_t *h_idx;  /* host, m x (N - 1) */
    const double *h_vals;  /* host, m */
} tf_request;

typedef struct tf_req_stats {
    double latency_us;     /* submit -> result on the host */
    double queue_us;       /* submit -> batch launched */
    int32_t batch_size;    /* requests in its batch */
    int32_t status;        /* TF_OK; TF_E_NUMERIC (a non-positive pivot: the
                              row is 0); TF_E_DEVICE (a HIP call of its batch
                              failed: the row is NaN, tf_serve_last_error says
                              which call) */
} tf_req_stats;

typedef struct tf_serve_stats {
    int64_t completed, batches, busy_rejects, max_queue;
    double p50_us, p90_us, p99_us, p999_us, max_us, mean_us;
    double solves_per_s;   /* completed / (last completion - first submit) */
    double mean_batch;
    int64_t failed;        /* completed with TF_E_DEVICE */
} tf_serve_stats;

typedef struct tf_server tf_server;

void tf_serve_default_options(tf_serve_opts *opt);
/* Starts the scheduler and completion threads.  NULL opts = defaults.  The
 * server reads ctx's factors and allocates its slots through ctx (counted
 * against tf_options.mem_budget): close it before tf_destroy(ctx), and do not
 * change the factors while it serves. */
tf_status tf_serve_open(tf_ctx *ctx, const tf_serve_opts *opts, tf_server **out);
/* Copies the request (caller may free it on return).  TF_E_BUSY when the
 * queue is full; TF_E_INVALID for m < 0 or a request whose device bytes
 * exceed one slot's share of the budget.  Thread-safe. */
tf_status tf_serve_submit(tf_server *srv, const tf_request *req, uint64_t *ticket);
/* Blocks until the ticket's row is done; h_row host[K] (may be NULL), st may
 * be NULL.  A ticket can be waited once.  Returns the request's status
 * (tf_req_stats.status).  Each request's status is its own: a failed
 * neighbour in the same batch does not change it.  Thread-safe. */
tf_status tf_serve_wait(tf_server *srv, uint64_t ticket, double *h_row, tf_req_stats *st);
/* Load generator: submits reqs[i] at h_arrival_s[i] seconds after the call
 * (non-decreasing), retrying while the queue is full; tickets[i] receives
 * each ticket.  Returns once all are submitted. */
tf_status tf_serve_replay(tf_server *srv, int64_t nreq, const double *h_arrival_s,
                          const tf_request *reqs, uint64_t *tickets);
/* Latency percentiles over the requests completed since open (or reset). */
tf_status tf_serve_report(tf_server *srv, tf_serve_stats *out);
tf_status tf_serve_reset_stats(tf_server *srv);
/* Waits for queued and in-flight requests, then stops the threads. */
void tf_serve_close(tf_server *srv);
/* Message of the last batch that failed with TF_E_DEVICE ("" if none); the
 * string stays valid until the calling thread's next call of this function. */
const char *tf_serve_last_error(tf_server *srv);
/* Test hook: the next `nbatches` batches fail at their launch step as if
 * the fold-in launch had returned an error (no kernel runs for them, the
 * GPU is not disturbed), so that the error path can be exercised.
 * TF_E_INVALID for nbatches < 0. */
tf_status tf_serve_inject_fault(tf_server *srv, int32_t nbatches);

/* ------------------------------------------------------------------ */
/* Kernel timing: HIP events around every launch of the row-accumulation
 * kernel (the one that gathers factor rows and builds the Gram matrices). */
typedef struct tf_kstats {
    int64_t launches;       /* accumulation launches timed */
    double total_ms;        /* summed event time */
    double alg_bytes;       /* summed algorithmic bytes of those launches */
    int64_t sweeps;
    int64_t first_launches; /* of which first passes of a split (residual */
    double first_ms;        /*   brought up to date in the same walk)     */
    double first_bytes;
    int64_t graph_sweeps;   /* sweeps captured or replayed as a graph */
} tf_kstats;
tf_status tf_profile(tf_ctx *ctx, int32_t enable);        /* 1 on, 0 off; resets */
tf_status tf_profile_read(tf_ctx *ctx, tf_kstats *out);    /* synchronises */

/* ------------------------------------------------------------------ */
/* Measurement probe (not part of the method): the rate of random 128-byte
 * row gathers, the requests the row passes of a split are bound by.
 *   d_table  device, rows x 32 floats (128-byte rows)
 *   rows     1 <= rows <= 2^32
 *   waves    wavefronts launched, a multiple of 4 (>= 4); each half
 *            wavefront reads `steps` rows (a multiple of 32), chosen by a
 *            SplitMix64-style hash of (seed, wave, step, half)
 *   d_out    device, waves x 64 floats (one running sum per lane)
 *   ms       out: HIP-event time of the launch on `stream`
 * Gathers made: waves * 2 * steps rows.  Synchronises the stream.
 * TF_E_INVALID for a count outside these rules. */
tf_status tf_probe_gather(const void *d_table, int64_t rows, int64_t waves, int64_t steps,
                          uint64_t seed, float *d_out, void *stream, double *ms);

/* ------------------------------------------------------------------ */
/* Host-only row planner (no GPU needed): classifies the rows of one mode
 * from its CSR offsets, as tf_init does for every mode.
 *   rowptr host[I + 1]; strategy, lane_nnz, split_threshold, chunk_nnz as in
 *   tf_options.  Outputs counts: tasks (wavefront work units), split rows and
 *   chunks, and per-G row counts hist[7] for G = 1,2,4,...,64 lanes per row.
 */
typedef struct tf_plan_summary {
    int64_t tasks;
    int64_t split_rows;
    int64_t chunks;
    int64_t empty_rows;
    int64_t rows_by_lanes[7];
} tf_plan_summary;
tf_status tf_plan_rows(const int64_t *rowptr, int64_t I, int32_t strategy, int32_t lane_nnz,
                       int32_t split_threshold, int32_t chunk_nnz, tf_plan_summary *out);

#ifdef __cplusplus
}
#endif
#endif /* TF_SALS_H */
