// Internal declarations of the SALS / CDTF GPU library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tf.h"
#include "plan.h"

namespace tfk {

// ---------------------------------------------------------------- precision
enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

struct bf16 {
    uint16_t bits;
};

// Largest number of columns per split: 16 for the register kernels (all
// precisions), 32 for the wide kernels (FP32 and BF16 storage).
constexpr int kMaxC = 32;
constexpr int kMaxModes = 8;
// Words of the failure flags after the per-mode failing rows (see pass_halted).
constexpr int kStopWord = kMaxModes;
constexpr int kCountWord = kMaxModes + 1;
constexpr int kWorkWord = kMaxModes + 2;   // task counter of persistent launches
constexpr int kFlagWords = kMaxModes + 3;

// Gram record of one row: upper triangle of B (c1 <= c2, row-major) then the
// right-hand side c; padded to a multiple of 4 entries.
__host__ __device__ constexpr int gram_entries(int CP) { return CP * (CP + 1) / 2 + CP; }
__host__ __device__ constexpr int gram_stride(int CP) { return (gram_entries(CP) + 3) & ~3; }

// ---------------------------------------------------------------- work plan
// (Task, Chunk, HostPlan, plan_rows, pick_cp: plan.h)

// ---------------------------------------------------------------- kernel args
struct AccumArgs {
    const int32_t *rowptr;
    const Task *tasks;
    int32_t ntasks;
    const int32_t *items;
    const Chunk *chunks;
    const int32_t *oidx[kMaxModes - 1];  // other modes ascending, CSR order
    void *rhat;                          // residual copy of this mode (CSR order)
    const int32_t *rperm;                // non-null (plain passes only): the
                                         // residual of entry j is rhat[rperm[j]]
    const void *W[kMaxModes - 1];        // other modes: current slabs
    const void *S[kMaxModes - 1];        // other modes: split-start slabs
    const void *P[kMaxModes - 1];        // other modes: pending-column slabs
    int32_t before[kMaxModes - 1];       // 1: that mode was updated earlier in this split
    const void *Sown;                    // this mode: split-start slab
    const void *Pown;                    // this mode: pending-column slab
    int32_t has_pend;
    int32_t no;                          // number of other modes (N - 1)
    int64_t ld;                          // slab row stride (elements)
    void *gram;                          // per-row Gram records
    void *gpart;                         // per-chunk partial Gram records
    unsigned int *work;                  // non-null: persistent launch, tasks taken
                                         // from this counter (zero at launch)
};

struct SolveArgs {
    const int32_t *rowptr;
    int64_t I;
    const void *gram;
    void *W;            // slab of the mode being updated
    int64_t ld;
    double lambda;
    int32_t reg_mode;
    unsigned long long *bad;   // smallest failing row (init ULLONG_MAX)
    unsigned long long *flags; // failure flags of the sweep (bad == flags + mode)
    int32_t nmodes;
};

// Workgroup-per-row path for splits wider than the register and wide kernels
// take (k_big.hip), up to kMaxBigC columns.
constexpr int kMaxBigC = 128;
constexpr int kColRingSlots = 64;   // pinned staging slots for split column lists (at least)
struct BigArgs {
    const int32_t *rowptr;               // this mode
    const int32_t *items;                // non-empty rows that are not chunked
    int32_t nitems;
    const int32_t *split_rows;           // chunked rows, and their chunk ranges
    const int32_t *split_chunk_ptr;
    int32_t nsplit;
    const int32_t *empty;                // rows with no entries
    int32_t nempty;
    const Chunk *chunks;
    int32_t nchunks;
    const int32_t *oidx[kMaxModes - 1];  // other modes ascending, CSR order
    const void *rhat;                    // mode 0's residual copy (R-hat of the split)
    const int32_t *rperm;                // non-null: entry q reads rhat[rperm[q]]
    const void *A[kMaxModes - 1];        // other modes' factors (storage type)
    void *Aown;                          // this mode's factor
    int32_t K;
    const int32_t *cols;                 // the split's columns (device, C)
    int32_t C;
    int32_t no;                          // N - 1
    void *gpart;                         // chunk records, big_record_stride(C) each
    double lambda;
    int32_t reg_mode;
    unsigned long long *bad;
    unsigned long long *flags;
    int32_t nmodes;
};
struct BoundaryArgs {
    void *r;                             // mode 0's residual copy (CSR order)
    const int32_t *perm;                 // mode 0's CSR order: entry of each position
    const int32_t *idx;                  // input-order index tuples (nnz x N)
    const void *A[kMaxModes];
    int32_t N, K;
    int64_t nnz;
    const int32_t *add;                  // columns added back (R-hat of the split)
    int32_t nadd;
    const int32_t *sub;                  // pending columns taken out (eq. (SALS_R))
    int32_t nsub;
};
hipError_t launch_big_pass(int prec, const BigArgs &a, hipStream_t st);
hipError_t launch_big_boundary(int prec, const BoundaryArgs &a, hipStream_t st);
int64_t big_record_stride(int C);

// launchers (return hipError_t of the launch)
hipError_t launch_accum(int prec, int CP, int no, bool first, const AccumArgs &a, int grid,
                        hipStream_t st);
hipError_t launch_solve(int prec, int CP, const SolveArgs &a, hipStream_t st);
hipError_t launch_clear_word(unsigned int *p, hipStream_t st);
hipError_t launch_pass_latch(unsigned long long *flags, int nmodes, hipStream_t st);
hipError_t launch_chunk_reduce(int prec, int CP, const int32_t *split_rows,
                               const int32_t *split_chunk_ptr, int nsplit, const void *gpart,
                               void *gram, hipStream_t st);

// ---------------------------------------------------------------- build kernels
hipError_t validate_input(const int32_t *idx, const double *vals, int64_t nnz, int N,
                          const int64_t *dims, unsigned long long *bad_idx,
                          unsigned long long *bad_val, hipStream_t st);
// stable sort of entry ids by key (keys < 2^bits); tmp buffers of nnz each
hipError_t stable_sort_by_key(const int32_t *idx, int N, int mode, int64_t nnz, int key_bits,
                              int32_t *perm_out, int32_t *k0, int32_t *k1, int32_t *v1,
                              int32_t *hist, int64_t hist_cap, int32_t *scan_tmp,
                              int64_t scan_tmp_cap, hipStream_t st);
int64_t sort_hist_size(int64_t nnz);
int64_t scan_tmp_size(int64_t n);
hipError_t rowptr_from_sorted(const int32_t *sorted_keys, int64_t nnz, int64_t I, int32_t *rowptr,
                              hipStream_t st);
hipError_t gather_other_index(const int32_t *idx, int N, int l, const int32_t *perm, int64_t nnz,
                              int32_t *out, hipStream_t st);
hipError_t init_factor(int prec, void *A, int64_t I, int K, uint64_t seed, uint64_t offset,
                       bool zero, hipStream_t st);
hipError_t residual_input_order(int prec, const int32_t *idx, const double *x, int64_t nnz,
                                int N, const void *const *A, int K, bool zero_model,
                                double *r_out, hipStream_t st);
hipError_t compose_with_mode0(const int32_t *perm0, const int32_t *permn, int64_t nnz,
                              int32_t *inv_scratch, int32_t *out, hipStream_t st);
hipError_t gather_copy(int prec, const void *in, const int32_t *idx, int64_t nnz, void *out,
                       hipStream_t st);
hipError_t gather_residual(int prec, const double *r_in, const int32_t *perm, int64_t nnz,
                           void *rhat_out, hipStream_t st);
hipError_t factor_to_f64(int prec, const void *A, int64_t n, double *out, hipStream_t st);
hipError_t factor_block_to_f64(int prec, const void *A, int K, const int32_t *rows,
                               int64_t nrows, const int32_t *cols, int ncols, double *out,
                               hipStream_t st);
hipError_t factor_from_f64(int prec, const double *in, int64_t n, void *A, hipStream_t st);

// ---------------------------------------------------------------- slabs
hipError_t pack_slab(int prec, const void *A, int64_t I, int K, const int32_t *cur, int ncur,
                     const int32_t *pend, int npend, int64_t sw, int64_t ld, void *Z, hipStream_t st);
hipError_t unpack_slab(int prec, const void *W, int64_t I, int K, const int32_t *cols, int ncols,
                       int64_t ld, void *A, hipStream_t st);

// ---------------------------------------------------------------- evaluation
struct EvalArgs {
    const int32_t *rowptr;   // mode 0
    const Task *tasks;
    int32_t ntasks;
    const int32_t *items;
    const Chunk *chunks;
    const int32_t *oidx[kMaxModes - 1];
    const void *rhat;        // mode-0 copy
    const void *P[kMaxModes - 1];  // pending-column slabs of the other modes
    const void *Pown;              // pending-column slab of mode 0
    int32_t npend;
    int32_t no;
    int64_t ld;
    const int32_t *perm;     // mode-0 CSR perm (for scatter to input order)
    double *r_out;           // if non-null: residual in input order
    double *partials;        // per-block sum of r^2
};
hipError_t launch_eval_residual(int prec, const EvalArgs &a, int grid, hipStream_t st);
hipError_t reg_partials(int prec, const void *A, int64_t I, int K, const int32_t *rowptr,
                        int weighted, double *partials, int nblocks, hipStream_t st);
hipError_t sum_partials(const double *partials, int64_t n, double *out, hipStream_t st);
hipError_t launch_predict(int prec, int N, int K, const void *const *A, const int64_t *dims,
                          const int32_t *q, int64_t m, double *out,
                          unsigned long long *bad, hipStream_t st);

}  // namespace tfk

// ---------------------------------------------------------------- context
struct tf_ctx {
    int N = 0;
    int64_t dims[tfk::kMaxModes] = {0};
    int64_t nnz = 0;
    int K = 0;
    double lambda = 0.0;
    tf_options opt{};
    int prec = 1;
    hipStream_t stream = nullptr;
    int device = 0;

    int32_t *idx = nullptr;   // nnz x N, input order
    double *x = nullptr;      // nnz, input order

    struct Mode {
        int64_t I = 0;
        int32_t *rowptr = nullptr;     // I + 1
        int32_t *perm = nullptr;       // nnz
        int32_t *oidx[tfk::kMaxModes - 1] = {nullptr};
        void *rhat = nullptr;          // nnz (TR)
        void *A = nullptr;             // I x K (TS)
        void *Z = nullptr;             // interleaved slab rows [W | P | S], I x ld (TS)
        tfk::Task *tasks = nullptr;
        int32_t ntasks = 0;
        int32_t *items = nullptr;
        int32_t nitems = 0;
        int32_t *empty = nullptr;           // rows with no entries
        int32_t nempty = 0;
        tfk::Chunk *chunks = nullptr;
        int32_t nchunks = 0;
        int32_t *split_rows = nullptr;
        int32_t *split_chunk_ptr = nullptr;
        int32_t nsplit = 0;
        std::vector<int64_t> h_rowptr;
        int32_t lane_nnz = 0, split_threshold = 0, chunk_nnz = 0;   // plan in use
        bool persistent = false;        // passes as one resident grid taking tasks
        // residual source of this mode's passes (modes >= 1): its own copy,
        // or mode 0's copy read through pos0 (position in mode-0 order of
        // each entry of this mode's order)
        int32_t *pos0 = nullptr;        // nnz, built on first use
        bool shared = false;            // the last split read mode 0's copy
        bool fresh = true;              // own copy holds the current R-hat
    } m[tfk::kMaxModes];

    int64_t ld = 0;           // slab row stride (elements, 128-byte multiple)
    int64_t sw = 0;           // slab segment width (elements)
    int slab_cp = 0;          // compute width the Gram buffers are sized for
    int64_t gpart_chunks = 0; // chunk records the partial buffer holds
    int tuned_C = 0;          // chosen by tf_autotune (0: none)
    void *gram = nullptr;     // max_I x gram_stride(slab_cp) (TA)
    void *gpart = nullptr;    // max_chunks x gram_stride(slab_cp) (TA)
    size_t gpart_bytes = 0;   // its size
    int32_t *d_cols = nullptr;  // device copy of split columns + pending columns
    int32_t *h_ring = nullptr;  // pinned staging slots for d_cols (ring_slots x (2K + 2))
    int ring_slots = 0;
    int ring_next = 0;
    unsigned long long *d_bad = nullptr;  // kFlagWords failure flags (pass_halted)
    double *d_partials = nullptr;
    int64_t partials_cap = 0;
    double *d_scalar = nullptr;

    std::vector<int32_t> order;     // column order for sweeps
    std::vector<int32_t> pend;      // columns whose contribution is pending in the copies
    bool stale = false;             // factors set without resync
    bool dirty = false;             // a numeric failure left the state inconsistent

    bool profiling = false;
    std::vector<hipEvent_t> ev_free;
    struct Timed { hipEvent_t a, b; double bytes; bool first; };
    std::vector<Timed> ev_pending;
    tf_kstats kstats{};
    int64_t sweeps_run = 0;         // tf_sweep calls (keys the random column orders)
    int auto_cp = 0;                // TF_STRATEGY_AUTO: width the tiles were tuned for

    // A sweep as one HIP graph (opt.graph).  Its device work depends on the
    // host state at its start only through the sizes, flags and buffers in
    // sweep_signature; the column lists it copies are rebuilt in their
    // pinned slots before each replay from where they came from: a range of
    // the column order, or the sweep's starting pending list.
    struct ColSrc { int kind = 0, begin = 0, len = 0; };   // 0 none, 1 order, 2 starting pend
    struct Upload { ColSrc cur, pend; };
    ColSrc pend_src;                // where pend came from (kept while capturing)
    bool capturing = false, capture_bad = false;
    std::vector<Upload> recipe;     // the captured sweep's column uploads, one per slot
    std::vector<int64_t> graph_sig, last_sig;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t own_stream = nullptr;   // created when a graph is asked for without a stream
    ColSrc graph_end_pend;          // pend after the captured sweep
    std::vector<char> graph_end_flags;  // shared, fresh per mode after it
    int64_t graph_end_ld = 0, graph_end_sw = 0;   // slab geometry after it

    // device memory of the context (ctx_alloc / ctx_free): the caller's hooks
    // or hipMalloc, counted against opt.mem_budget
    std::mutex mem_mu;
    std::unordered_map<void *, size_t> mem_live;
    size_t mem_bytes = 0;

    std::string err;
};

// Device allocation for a context (see tf_options.mem_budget / dev_alloc):
// hipErrorOutOfMemory when the budget or the allocator refuses.
hipError_t ctx_alloc(tf_ctx *c, void **p, size_t bytes);
void ctx_free(tf_ctx *c, void *p);
