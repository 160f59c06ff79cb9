// C ABI of the SALS / CDTF GPU path: context construction, the split driver
// of Algorithm 1 (arXiv:1410.5209), loss, prediction and state access.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "foldin.h"
#include "tf_internal.h"

using namespace tfk;

namespace tfk {
hipError_t launch_accum_f64(int CP, int no, bool first, const AccumArgs &a, int grid, hipStream_t st);
hipError_t launch_accum_f32(int CP, int no, bool first, const AccumArgs &a, int grid, hipStream_t st);
hipError_t launch_accum_bf16(int CP, int no, bool first, const AccumArgs &a, int grid, hipStream_t st);
hipError_t launch_solve_f64(int CP, const SolveArgs &a, hipStream_t st);
hipError_t launch_solve_f32(int CP, const SolveArgs &a, hipStream_t st);
hipError_t launch_solve_bf16(int CP, const SolveArgs &a, hipStream_t st);
hipError_t launch_reduce_f64(int CP, const int32_t *, const int32_t *, int, const void *, void *, hipStream_t);
hipError_t launch_reduce_f32(int CP, const int32_t *, const int32_t *, int, const void *, void *, hipStream_t);
hipError_t launch_reduce_bf16(int CP, const int32_t *, const int32_t *, int, const void *, void *, hipStream_t);

hipError_t launch_accum(int prec, int CP, int no, bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    if (prec == P_F64) return launch_accum_f64(CP, no, first, a, grid, st);
    if (prec == P_F32) return launch_accum_f32(CP, no, first, a, grid, st);
    return launch_accum_bf16(CP, no, first, a, grid, st);
}
hipError_t launch_solve(int prec, int CP, const SolveArgs &a, hipStream_t st)
{
    if (prec == P_F64) return launch_solve_f64(CP, a, st);
    if (prec == P_F32) return launch_solve_f32(CP, a, st);
    return launch_solve_bf16(CP, a, st);
}
hipError_t launch_chunk_reduce(int prec, int CP, const int32_t *rows, const int32_t *ptr, int nsplit,
                               const void *gpart, void *gram, hipStream_t st)
{
    if (prec == P_F64) return launch_reduce_f64(CP, rows, ptr, nsplit, gpart, gram, st);
    if (prec == P_F32) return launch_reduce_f32(CP, rows, ptr, nsplit, gpart, gram, st);
    return launch_reduce_bf16(CP, rows, ptr, nsplit, gpart, gram, st);
}
}  // namespace tfk

hipError_t ctx_alloc(tf_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    {
        std::lock_guard<std::mutex> g(c->mem_mu);
        if (c->opt.mem_budget && c->mem_bytes + bytes > c->opt.mem_budget) return hipErrorOutOfMemory;
        c->mem_bytes += bytes;  // reserved while the allocator runs
    }
    void *q = nullptr;
    hipError_t e = hipSuccess;
    if (c->opt.dev_alloc) {
        q = c->opt.dev_alloc(bytes, c->opt.stream, c->opt.alloc_user);
        if (!q) e = hipErrorOutOfMemory;
        else if (reinterpret_cast<uintptr_t>(q) & 255) {
            c->opt.dev_free(q, bytes, c->opt.stream, c->opt.alloc_user);
            q = nullptr;
            e = hipErrorInvalidValue;
        }
    } else {
        e = hipMalloc(&q, bytes);
    }
    std::lock_guard<std::mutex> g(c->mem_mu);
    if (e != hipSuccess) {
        c->mem_bytes -= bytes;
        return e;
    }
    c->mem_live[q] = bytes;
    *p = q;
    return hipSuccess;
}

void ctx_free(tf_ctx *c, void *p)
{
    if (!p) return;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> g(c->mem_mu);
        auto it = c->mem_live.find(p);
        if (it == c->mem_live.end()) return;  // not this context's block
        bytes = it->second;
        c->mem_live.erase(it);
        c->mem_bytes -= bytes;
    }
    if (c->opt.dev_free) c->opt.dev_free(p, bytes, c->opt.stream, c->opt.alloc_user);
    else (void)hipFree(p);
}

namespace {

thread_local std::string g_init_err;

size_t ts_size(int prec) { return prec == P_F64 ? 8 : (prec == P_F32 ? 4 : 2); }
size_t tr_size(int prec) { return prec == P_F64 ? 8 : 4; }
size_t ta_size(int prec) { return prec == P_F64 ? 8 : 4; }
int vec_w(int prec) { return (int)(16 / ts_size(prec)); }

tf_status set_err(std::string *dst, tf_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    *dst = buf;
    return s;
}

#define CTX_FAIL(ctx, s, ...) set_err(&(ctx)->err, (s), __VA_ARGS__)
#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return CTX_FAIL(ctx, e_ == hipErrorOutOfMemory ? TF_E_NOMEM : TF_E_DEVICE,     \
                            "%s failed: %s", #call, hipGetErrorString(e_));                \
    } while (0)

template <typename T>
hipError_t dalloc(tf_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    const hipError_t e = ctx_alloc(c, &q, (count ? count : 1) * sizeof(T));
    *p = static_cast<T *>(q);
    return e;
}

void dfree(tf_ctx *c, void *p) { ctx_free(c, p); }

int key_bits_for(int64_t I)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < I) ++b;
    return b;
}

// Ensure the Gram buffers hold records of compute width CP.
tf_status ensure_gram(tf_ctx *c, int CP)
{
    int64_t maxI = 0, maxch = 1;
    for (int n = 0; n < c->N; ++n) {
        maxI = std::max<int64_t>(maxI, c->m[n].I);
        maxch = std::max<int64_t>(maxch, c->m[n].nchunks);
    }
    if (CP <= c->slab_cp && c->gram && maxch <= c->gpart_chunks) return TF_OK;
    const int cp = std::max(CP, c->slab_cp);
    dfree(c, c->gram);
    dfree(c, c->gpart);
    c->gram = c->gpart = nullptr;
    const size_t rec = (size_t)gram_stride(cp) * ta_size(c->prec);
    HIPCHK(c, ctx_alloc(c, &c->gram, (size_t)maxI * rec));
    HIPCHK(c, ctx_alloc(c, &c->gpart, (size_t)maxch * rec));
    c->gpart_bytes = (size_t)maxch * rec;
    c->slab_cp = cp;
    c->gpart_chunks = maxch;
    return TF_OK;
}

// Chunk records of the workgroup-per-row path for C columns.
tf_status ensure_gpart_big(tf_ctx *c, int C)
{
    int64_t maxch = 1;
    for (int n = 0; n < c->N; ++n) maxch = std::max<int64_t>(maxch, c->m[n].nchunks);
    const size_t need = (size_t)maxch * (size_t)big_record_stride(C) * ta_size(c->prec);
    if (c->gpart && c->gpart_bytes >= need) return TF_OK;
    dfree(c, c->gpart);
    c->gpart = nullptr;
    c->gpart_bytes = 0;
    c->gpart_chunks = 0;   // the narrow path re-sizes it for its records
    HIPCHK(c, ctx_alloc(c, &c->gpart, need));
    c->gpart_bytes = need;
    return TF_OK;
}

// Bytes reserved per slab row: three segments of up to kMaxC elements plus
// alignment, rounded to whole 128-byte lines.
constexpr size_t kSlabRowBytes = 384;

// Segment width and row stride of the interleaved slabs for a given number
// of columns: segments of whole 8-byte units (so W and S start 16-byte
// aligned), rows padded to whole 128-byte lines so that no row straddles a
// line it does not need.  (Keeping W, P and S in three separate arrays
// instead, once a segment fills whole lines, was measured on the 5-way
// workload at C = 32 and changed no pass time.)
tf_status slab_geometry(tf_ctx *c, int width)
{
    const int64_t q = c->prec == P_BF16 ? 4 : 2;
    const int64_t sw = (std::max(width, 1) + q - 1) / q * q;
    const int64_t vw = vec_w(c->prec);
    const int64_t need = std::max<int64_t>(3 * sw, 2 * sw + (sw + vw - 1) / vw * vw);
    const int64_t per_line = 128 / (int64_t)ts_size(c->prec);
    const int64_t lines = (need + per_line - 1) / per_line;
    if (lines * 128 > (int64_t)kSlabRowBytes)
        return CTX_FAIL(c, TF_E_UNSUPPORTED, "slab row of %lld lines exceeds the allocation",
                        (long long)lines);
    c->sw = sw;
    c->ld = lines * per_line;
    return TF_OK;
}

const void *seg(const tf_ctx *c, const void *Z, int which)
{
    return static_cast<const char *>(Z) + (size_t)which * (size_t)c->sw * ts_size(c->prec);
}

void fill_accum_args(tf_ctx *c, int n, int npend, AccumArgs *a)
{
    std::memset(a, 0, sizeof *a);
    auto &md = c->m[n];
    a->rowptr = md.rowptr;
    a->tasks = md.tasks;
    a->ntasks = md.ntasks;
    a->items = md.items;
    a->chunks = md.chunks;
    a->rhat = md.rhat;
    int t = 0;
    for (int l = 0; l < c->N; ++l) {
        if (l == n) continue;
        a->oidx[t] = md.oidx[t];
        a->W[t] = seg(c, c->m[l].Z, 0);
        a->P[t] = seg(c, c->m[l].Z, 1);
        a->S[t] = seg(c, c->m[l].Z, 2);
        a->before[t] = l < n ? 1 : 0;
        ++t;
    }
    a->Pown = seg(c, md.Z, 1);
    a->Sown = seg(c, md.Z, 2);
    a->has_pend = npend > 0 ? 1 : 0;
    a->no = c->N - 1;
    a->ld = c->ld;
    a->gram = c->gram;
    a->gpart = c->gpart;
    a->work = md.persistent ? reinterpret_cast<unsigned int *>(c->d_bad + kWorkWord) : nullptr;
}

// The work counter of a persistent launch starts at zero (a stream-ordered
// clear before each launch, by a kernel: a captured sweep holds no memset).
tf_status reset_work(tf_ctx *c, const AccumArgs &a)
{
    if (a.work) HIPCHK(c, launch_clear_word(a.work, c->stream));
    return TF_OK;
}

hipEvent_t take_event(tf_ctx *c)
{
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Algorithmic bytes of one accumulation launch (design-neutral byte model:
// every index, residual and gathered factor element read once per use, no
// cache credit).  Row pass: per entry 4(N-1) index bytes, one residual read,
// (N-1) C factor elements; per row one offset.  The first pass of a split
// also carries 1/N of the split's residual work (R-hat and eq. (SALS_R) done
// once on a single residual array: per entry 4N index bytes, a residual read
// and write, N (C_prev + C) factor elements).
double alg_bytes(const tf_ctx *c, int n, int C, int npend, bool first)
{
    const double N = c->N, sf = (double)ts_size(c->prec), sr = (double)tr_size(c->prec);
    const double nnz = (double)c->nnz;
    double b = nnz * (4.0 * (N - 1) + sr + (N - 1) * C * sf) + 4.0 * (double)(c->m[n].I + 1);
    if (first) b += nnz * (4.0 * N + 2.0 * sr + N * (npend + C) * sf) / N;
    return b;
}

tf_status pack_all(tf_ctx *c, const int32_t *d_cur, int ncur, const int32_t *d_pend, int npend)
{
    for (int l = 0; l < c->N; ++l) {
        auto &md = c->m[l];
        hipError_t e = pack_slab(c->prec, md.A, md.I, c->K, d_cur, ncur, d_pend, npend, c->sw,
                                 c->ld, md.Z, c->stream);
        if (e != hipSuccess) return CTX_FAIL(c, TF_E_DEVICE, "pack: %s", hipGetErrorString(e));
    }
    return TF_OK;
}

// Upload the current columns (offset 0) and the pending columns (offset K).
// The host side goes through a ring of pinned slots, so a sweep is queued
// without waiting for the GPU: the copy out of a slot is ordered after the
// kernels that read the previous list, and a slot is written again only
// after the stream has drained (when the ring wraps).
tf_status ensure_ring(tf_ctx *c, int slots)
{
    slots = std::max(slots, kColRingSlots);
    if (c->h_ring && c->ring_slots >= slots) return TF_OK;
    if (c->h_ring) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipHostFree(c->h_ring));
        c->h_ring = nullptr;
    }
    const size_t slot = 2 * (size_t)c->K + 2;
    HIPCHK(c, hipHostMalloc(reinterpret_cast<void **>(&c->h_ring), (size_t)slots * slot * sizeof(int32_t),
                            hipHostMallocDefault));
    c->ring_slots = slots;
    c->ring_next = 0;
    return TF_OK;
}

// Where a column list handed to upload_cols lives, for replays of a
// captured sweep: a range of the column order, or (see tf_sweep) the
// sweep's starting pending list.
tf_ctx::ColSrc col_source(const tf_ctx *c, const int32_t *cols, int ncols)
{
    tf_ctx::ColSrc s;
    if (ncols == 0) return s;
    const int32_t *o = c->order.data();
    if (cols >= o && cols + ncols <= o + c->order.size()) {
        s.kind = 1;
        s.begin = (int)(cols - o);
        s.len = ncols;
    } else {
        s.kind = -1;   // not reproducible from the order
    }
    return s;
}

void fill_slot(const tf_ctx *c, int32_t *h, const int32_t *cols, int ncols, const int32_t *pend,
               int npend)
{
    std::fill(h, h + 2 * (size_t)c->K + 2, 0);
    for (int q = 0; q < ncols; ++q) h[q] = cols[q];
    for (int q = 0; q < npend; ++q) h[c->K + q] = pend[q];
}

tf_status upload_cols(tf_ctx *c, const int32_t *cols, int ncols)
{
    const size_t slot = 2 * (size_t)c->K + 2;
    tf_status s = ensure_ring(c, kColRingSlots);
    if (s != TF_OK) return s;
    if (c->ring_next == c->ring_slots) {
        if (c->capturing) {   // no waiting inside a capture: the sweep runs eagerly instead
            c->capture_bad = true;
            return CTX_FAIL(c, TF_E_STATE, "column slots exhausted while capturing");
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->ring_next = 0;
    }
    if (c->capturing) {
        tf_ctx::Upload u{col_source(c, cols, ncols), c->pend_src};
        if (u.cur.kind < 0 || u.pend.kind < 0) c->capture_bad = true;
        c->recipe.push_back(u);
    }
    int32_t *h = c->h_ring + (size_t)c->ring_next++ * slot;
    fill_slot(c, h, cols, ncols, c->pend.data(), (int)c->pend.size());
    HIPCHK(c, hipMemcpyAsync(c->d_cols, h, slot * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    return TF_OK;
}

// 128-byte lines a pass touches in one gathered slab row: the W segment,
// plus P and S when asked (each segment read over CP columns).
int row_lines(const tf_ctx *c, int CP, bool p, bool s)
{
    const int64_t sf = (int64_t)ts_size(c->prec), seg_b = c->sw * sf, len = CP * sf;
    bool used[8] = {false};
    auto mark = [&](int k) {
        for (int64_t b = k * seg_b; b < k * seg_b + len; b += 8) used[std::min<int64_t>(b / 128, 7)] = true;
    };
    mark(0);
    if (p) mark(1);
    if (s) mark(2);
    int n = 0;
    for (bool u : used) n += u ? 1 : 0;
    return n;
}

// Whether mode n (>= 1) reads mode 0's residual copy in this split: the
// option, or (auto) the smaller count of random line requests per entry
// over the split's T_in passes.  Own copy: the first pass gathers W, P (when
// columns are pending) and S (modes already updated) of every other mode,
// and is charged one line more for writing the residual back and for the
// boundary arithmetic (measured: a first pass costs more than its gathers).
// Shared: W only, plus one residual read per pass.  Ties go to shared.
bool want_shared(const tf_ctx *c, int n, int CP, int npend, int T_in)
{
    if (n == 0 || c->opt.resid_share == TF_RESID_OWN) return false;
    if (c->opt.resid_share == TF_RESID_SHARED) return true;
    int own = 1, shared = T_in;
    for (int l = 0; l < c->N; ++l) {
        if (l == n) continue;
        const int w = row_lines(c, CP, false, false);
        own += row_lines(c, CP, npend > 0, l < n) + (T_in - 1) * w;
        shared += T_in * w;
    }
    return shared <= own;
}

// pos0 of mode n: position in mode 0's order of each entry of mode n's order.
tf_status ensure_pos0(tf_ctx *c, int n)
{
    auto &md = c->m[n];
    if (md.pos0) return TF_OK;
    int32_t *inv = nullptr;
    HIPCHK(c, dalloc(c, &md.pos0, (size_t)c->nnz));
    HIPCHK(c, dalloc(c, &inv, (size_t)c->nnz));
    hipError_t e = compose_with_mode0(c->m[0].perm, md.perm, c->nnz, inv, md.pos0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, inv);
    if (e != hipSuccess) return CTX_FAIL(c, TF_E_DEVICE, "pos0: %s", hipGetErrorString(e));
    return TF_OK;
}

// Residual sources for a split; a mode returning to its own copy first takes
// mode 0's R-hat of the previous split (the value its copy would hold).
tf_status place_residuals(tf_ctx *c, int CP, int npend, int T_in)
{
    for (int n = 1; n < c->N; ++n) {
        auto &md = c->m[n];
        const bool sh = want_shared(c, n, CP, npend, T_in);
        if (sh) {
            tf_status s = ensure_pos0(c, n);
            if (s != TF_OK) return s;
        } else if (!md.fresh) {
            HIPCHK(c, gather_copy(c->prec, c->m[0].rhat, md.pos0, c->nnz, md.rhat, c->stream));
            md.fresh = true;
        }
        md.shared = sh;
    }
    return TF_OK;
}

// Mode 0's residual copy brought to R-hat of the columns `add` with the
// pending columns' eq. (SALS_R) applied (k_big_boundary, from the factors,
// which hold the pending columns' final values).  The other modes' own
// copies no longer match it: they take it again through pos0 when next
// used.  Clears the pending list.
tf_status boundary_on_mode0(tf_ctx *c, const int32_t *d_add, int nadd)
{
    BoundaryArgs b;
    std::memset(&b, 0, sizeof b);
    b.r = c->m[0].rhat;
    b.perm = c->m[0].perm;
    b.idx = c->idx;
    for (int n = 0; n < c->N; ++n) b.A[n] = c->m[n].A;
    b.N = c->N;
    b.K = c->K;
    b.nnz = c->nnz;
    b.add = d_add;
    b.nadd = nadd;
    b.sub = c->d_cols + c->K;
    b.nsub = (int)c->pend.size();
    HIPCHK(c, launch_big_boundary(c->prec, b, c->stream));
    for (int n = 1; n < c->N; ++n) c->m[n].fresh = false;
    c->pend.clear();
    c->pend_src = tf_ctx::ColSrc{};
    return TF_OK;
}

// Take the pending columns out of the residual before a pass that cannot
// carry them (too many for its slab segments).
tf_status flush_pending(tf_ctx *c)
{
    if (c->pend.empty()) return TF_OK;
    tf_status s = upload_cols(c, nullptr, 0);
    if (s != TF_OK) return s;
    return boundary_on_mode0(c, c->d_cols, 0);
}

// A split wider than the narrow kernels take (k_big.hip): R-hat formed on
// mode 0's copy, every mode reading that copy, factor rows updated in place.
tf_status run_split_big(tf_ctx *c, const int32_t *cols, int ncols, int T_in)
{
    tf_status s = ensure_gpart_big(c, ncols);
    if (s != TF_OK) return s;
    if ((s = upload_cols(c, cols, ncols)) != TF_OK) return s;
    if ((s = boundary_on_mode0(c, c->d_cols, ncols)) != TF_OK) return s;
    for (int n = 1; n < c->N; ++n) {
        if ((s = ensure_pos0(c, n)) != TF_OK) return s;
        c->m[n].shared = true;
    }
    for (int it = 0; it < T_in; ++it) {
        for (int n = 0; n < c->N; ++n) {
            auto &md = c->m[n];
            BigArgs a;
            std::memset(&a, 0, sizeof a);
            a.rowptr = md.rowptr;
            a.items = md.items;
            a.nitems = md.nitems;
            a.split_rows = md.split_rows;
            a.split_chunk_ptr = md.split_chunk_ptr;
            a.nsplit = md.nsplit;
            a.empty = md.empty;
            a.nempty = md.nempty;
            a.chunks = md.chunks;
            a.nchunks = md.nchunks;
            int t = 0;
            for (int l = 0; l < c->N; ++l) {
                if (l == n) continue;
                a.oidx[t] = md.oidx[t];
                a.A[t] = c->m[l].A;
                ++t;
            }
            a.rhat = c->m[0].rhat;
            a.rperm = n > 0 ? md.pos0 : nullptr;
            a.Aown = md.A;
            a.K = c->K;
            a.cols = c->d_cols;
            a.C = ncols;
            a.no = c->N - 1;
            a.gpart = c->gpart;
            a.lambda = c->lambda;
            a.reg_mode = c->opt.reg_mode;
            a.bad = c->d_bad + n;
            a.flags = c->d_bad;
            a.nmodes = c->N;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (c->profiling) {
                e0 = take_event(c);
                e1 = take_event(c);
                if (e0) HIPCHK(c, hipEventRecord(e0, c->stream));
            }
            HIPCHK(c, launch_big_pass(c->prec, a, c->stream));
            if (c->profiling && e0 && e1) {
                HIPCHK(c, hipEventRecord(e1, c->stream));
                c->ev_pending.push_back(tf_ctx::Timed{e0, e1, alg_bytes(c, n, ncols, 0, false), false});
            }
            HIPCHK(c, launch_pass_latch(c->d_bad, c->N, c->stream));
        }
    }
    c->pend.assign(cols, cols + ncols);
    c->pend_src = col_source(c, cols, ncols);
    return TF_OK;
}

// One split of Algorithm 1 on columns cols[0..ncols).
tf_status run_split(tf_ctx *c, const int32_t *cols, int ncols, int T_in)
{
    if (pick_cp(ncols, c->prec) < 0) return run_split_big(c, cols, ncols, T_in);
    // pending columns too many for this split's slab segments (after a wider
    // split) are taken out of the residual first
    if (pick_cp(std::max<int>(ncols, (int)c->pend.size()), c->prec) < 0) {
        tf_status s0 = flush_pending(c);
        if (s0 != TF_OK) return s0;
    }
    // the kernels run at a width covering both this split's and the pending
    // columns, so the residual update stays fused into the first pass (the
    // padded columns are zero in every slab segment, which leaves the real
    // columns' solution unchanged and the padded ones at zero)
    int CP = pick_cp(std::max<int>(ncols, (int)c->pend.size()), c->prec);
    if (CP < 0) return CTX_FAIL(c, TF_E_UNSUPPORTED, "no kernel width for C = %d", ncols);
    tf_status s = ensure_gram(c, CP);
    if (s != TF_OK) return s;
    const int npend = (int)c->pend.size();
    if ((s = slab_geometry(c, std::max(CP, npend))) != TF_OK) return s;
    if ((s = upload_cols(c, cols, ncols)) != TF_OK) return s;
    const int32_t *d_cur = c->d_cols;
    const int32_t *d_pend = c->d_cols + c->K;

    if ((s = place_residuals(c, CP, npend, T_in)) != TF_OK) return s;

    // slabs at the start of the split: S (snapshot) and W (working copy) hold
    // the split's columns, P the previous split's columns (final values)
    if ((s = pack_all(c, d_cur, ncols, d_pend, npend)) != TF_OK) return s;

    for (int it = 0; it < T_in; ++it) {
        for (int n = 0; n < c->N; ++n) {
            auto &md = c->m[n];
            const bool first = it == 0;
            const bool sh = n > 0 && md.shared;
            AccumArgs a;
            fill_accum_args(c, n, first && !sh ? npend : 0, &a);
            if (sh) {
                a.rhat = c->m[0].rhat;
                a.rperm = md.pos0;
            }
            const int grid = (md.ntasks + 3) / 4;
            if (grid > 0) {
                tf_status s0 = reset_work(c, a);
                if (s0 != TF_OK) return s0;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->profiling) {
                    e0 = take_event(c);
                    e1 = take_event(c);
                    if (e0) HIPCHK(c, hipEventRecord(e0, c->stream));
                }
                HIPCHK(c, launch_accum(c->prec, CP, c->N - 1, first && !sh, a, grid, c->stream));
                if (c->profiling && e0 && e1) {
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    c->ev_pending.push_back(
                        tf_ctx::Timed{e0, e1, alg_bytes(c, n, ncols, npend, first), first});
                }
            }
            if (md.nsplit > 0)
                HIPCHK(c, launch_chunk_reduce(c->prec, CP, md.split_rows, md.split_chunk_ptr,
                                              md.nsplit, c->gpart, c->gram, c->stream));
            SolveArgs sa;
            sa.rowptr = md.rowptr;
            sa.I = md.I;
            sa.gram = c->gram;
            sa.W = md.Z;
            sa.ld = c->ld;
            sa.lambda = c->lambda;
            sa.reg_mode = c->opt.reg_mode;
            sa.bad = c->d_bad + n;
            sa.flags = c->d_bad;
            sa.nmodes = c->N;
            HIPCHK(c, launch_solve(c->prec, CP, sa, c->stream));
            HIPCHK(c, launch_pass_latch(c->d_bad, c->N, c->stream));
        }
    }
    for (int l = 0; l < c->N; ++l) {
        auto &md = c->m[l];
        HIPCHK(c, unpack_slab(c->prec, md.Z, md.I, c->K, d_cur, ncols, c->ld, md.A, c->stream));
        if (md.shared) md.fresh = false;
    }
    c->pend.assign(cols, cols + ncols);
    c->pend_src = col_source(c, cols, ncols);
    return TF_OK;
}

tf_status reset_bad(tf_ctx *c)
{
    HIPCHK(c, hipMemsetAsync(c->d_bad, 0xff, kMaxModes * sizeof(unsigned long long), c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_bad + kStopWord, 0, 2 * sizeof(unsigned long long), c->stream));
    return TF_OK;
}

tf_status check_bad(tf_ctx *c)
{
    unsigned long long h[kMaxModes];
    HIPCHK(c, hipMemcpyAsync(h, c->d_bad, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int n = 0; n < c->N; ++n)
        if (h[n] != ULLONG_MAX)
            return CTX_FAIL(c, TF_E_NUMERIC,
                            "non-positive Cholesky pivot in mode %d row %llu (row kept its previous value; "
                            "no factor was updated after that mode pass)",
                            n, (unsigned long long)h[n]);
    return TF_OK;
}

tf_status check_ready(tf_ctx *c)
{
    if (c->stale) return CTX_FAIL(c, TF_E_STATE, "factors were set; call tf_resync first");
    return TF_OK;
}

tf_status ensure_partials(tf_ctx *c, int64_t n)
{
    if (n <= c->partials_cap) return TF_OK;
    dfree(c, c->d_partials);
    c->d_partials = nullptr;
    HIPCHK(c, dalloc(c, &c->d_partials, (size_t)n));
    c->partials_cap = n;
    return TF_OK;
}

// Sum of r^2 over all entries (and optionally r in input order).
tf_status eval_residual(tf_ctx *c, double *d_rout, double *se_out)
{
    // the pending columns go into the W segment of the slabs; more than a
    // slab row holds (after a wide split) are taken out of the residual first
    if (pick_cp((int)c->pend.size(), c->prec) < 0) {
        tf_status s0 = flush_pending(c);
        if (s0 != TF_OK) return s0;
    }
    const int npend = (int)c->pend.size();
    tf_status s = slab_geometry(c, std::max(npend, 1));
    if (s != TF_OK) return s;
    if (npend > 0) {
        if ((s = upload_cols(c, c->pend.data(), npend)) != TF_OK) return s;
        if ((s = pack_all(c, c->d_cols, npend, c->d_cols, 0)) != TF_OK) return s;
    }
    auto &m0 = c->m[0];
    EvalArgs a;
    std::memset(&a, 0, sizeof a);
    a.rowptr = m0.rowptr;
    a.tasks = m0.tasks;
    a.ntasks = m0.ntasks;
    a.items = m0.items;
    a.chunks = m0.chunks;
    for (int l = 1; l < c->N; ++l) {
        a.oidx[l - 1] = m0.oidx[l - 1];
        a.P[l - 1] = c->m[l].Z;
    }
    a.rhat = m0.rhat;
    a.Pown = m0.Z;
    a.npend = npend;
    a.no = c->N - 1;
    a.ld = c->ld;
    a.perm = m0.perm;
    a.r_out = d_rout;
    const int grid = std::max(1, (m0.ntasks + 3) / 4);
    if ((s = ensure_partials(c, grid)) != TF_OK) return s;
    a.partials = c->d_partials;
    HIPCHK(c, launch_eval_residual(c->prec, a, grid, c->stream));
    HIPCHK(c, sum_partials(c->d_partials, grid, c->d_scalar, c->stream));
    double h = 0.0;
    HIPCHK(c, hipMemcpyAsync(&h, c->d_scalar, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *se_out = h;
    return TF_OK;
}

void destroy_ctx(tf_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    dfree(c, c->idx);
    dfree(c, c->x);
    for (int n = 0; n < kMaxModes; ++n) {
        auto &md = c->m[n];
        dfree(c, md.rowptr); dfree(c, md.perm);
        for (int l = 0; l < kMaxModes - 1; ++l) dfree(c, md.oidx[l]);
        dfree(c, md.rhat); dfree(c, md.A); dfree(c, md.Z);
        dfree(c, md.tasks); dfree(c, md.items); dfree(c, md.chunks);
        dfree(c, md.split_rows); dfree(c, md.split_chunk_ptr);
        dfree(c, md.pos0); dfree(c, md.empty);
    }
    dfree(c, c->gram); dfree(c, c->gpart); dfree(c, c->d_cols); dfree(c, c->d_bad);
    dfree(c, c->d_partials); dfree(c, c->d_scalar);
    if (c->h_ring) {   // no copy may still read it (also on the null stream)
        (void)hipStreamSynchronize(c->stream);
        (void)hipHostFree(c->h_ring);
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    for (auto &t : c->ev_pending) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
    delete c;
}

template <typename T>
tf_status upload_vec(tf_ctx *c, T **dst, const std::vector<T> &v)
{
    HIPCHK(c, dalloc(c, dst, v.size()));
    if (!v.empty())
        HIPCHK(c, hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TF_OK;
}

// Plan mode n's rows with the given tile parameters and upload the plan.
tf_status apply_plan(tf_ctx *c, int n, int lane_nnz, int split_threshold, int chunk_nnz)
{
    auto &md = c->m[n];
    HostPlan plan;
    const int strategy = c->opt.strategy == TF_STRATEGY_PLAIN ? TF_STRATEGY_PLAIN : TF_STRATEGY_SKEW;
    plan_rows(md.h_rowptr.data(), md.I, strategy, lane_nnz, split_threshold, chunk_nnz, &plan);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, md.tasks); dfree(c, md.items); dfree(c, md.chunks); dfree(c, md.split_rows); dfree(c, md.split_chunk_ptr);
    dfree(c, md.empty);
    md.tasks = nullptr; md.items = nullptr; md.chunks = nullptr;
    md.split_rows = nullptr; md.split_chunk_ptr = nullptr; md.empty = nullptr;
    tf_status s;
    if ((s = upload_vec(c, &md.tasks, plan.tasks)) != TF_OK) return s;
    if ((s = upload_vec(c, &md.items, plan.items)) != TF_OK) return s;
    if ((s = upload_vec(c, &md.chunks, plan.chunks)) != TF_OK) return s;
    if ((s = upload_vec(c, &md.split_rows, plan.split_rows)) != TF_OK) return s;
    if ((s = upload_vec(c, &md.split_chunk_ptr, plan.split_chunk_ptr)) != TF_OK) return s;
    if ((s = upload_vec(c, &md.empty, plan.empty)) != TF_OK) return s;
    md.nitems = (int32_t)plan.items.size();
    md.nempty = (int32_t)plan.empty.size();
    md.ntasks = (int32_t)plan.tasks.size();
    md.nchunks = (int32_t)plan.chunks.size();
    md.nsplit = (int32_t)plan.split_rows.size();
    md.lane_nnz = lane_nnz;
    md.split_threshold = split_threshold;
    md.chunk_nnz = chunk_nnz;
    return TF_OK;
}

tf_status build_state(tf_ctx *c, const int32_t *d_idx, const double *d_vals)
{
    const int N = c->N;
    const int64_t nnz = c->nnz;
    hipStream_t st = c->stream;
    HIPCHK(c, dalloc(c, &c->idx, (size_t)nnz * N));
    HIPCHK(c, dalloc(c, &c->x, (size_t)nnz));
    HIPCHK(c, hipMemcpyAsync(c->idx, d_idx, (size_t)nnz * N * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->x, d_vals, (size_t)nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(c, dalloc(c, &c->d_bad, kFlagWords));
    HIPCHK(c, dalloc(c, &c->d_scalar, 4));
    HIPCHK(c, dalloc(c, &c->d_cols, 2 * (size_t)c->K + 2));

    // validation: first bad index tuple and first non-finite value
    HIPCHK(c, hipMemsetAsync(c->d_bad, 0xff, 2 * sizeof(unsigned long long), st));
    HIPCHK(c, validate_input(c->idx, c->x, nnz, N, c->dims, c->d_bad, c->d_bad + 1, st));
    unsigned long long hb[2];
    HIPCHK(c, hipMemcpyAsync(hb, c->d_bad, sizeof hb, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (hb[0] != ULLONG_MAX)
        return CTX_FAIL(c, TF_E_INVALID, "entry %llu has an index outside its mode length", hb[0]);
    if (hb[1] != ULLONG_MAX)
        return CTX_FAIL(c, TF_E_INVALID, "entry %llu has a non-finite value", hb[1]);

    // CSR per mode (stable sort of entry ids by row)
    int32_t *k0 = nullptr, *k1 = nullptr, *v1 = nullptr, *hist = nullptr, *stmp = nullptr;
    const int64_t hcap = sort_hist_size(nnz);
    const int64_t scap = scan_tmp_size(hcap);
    struct Tmp { tf_ctx *c; int32_t **p; ~Tmp() { for (int i = 0; i < 5; ++i) dfree(c, p[i]); } };
    int32_t *tmps[5] = {nullptr};
    Tmp guard{c, tmps};
    HIPCHK(c, dalloc(c, &k0, (size_t)nnz)); tmps[0] = k0;
    HIPCHK(c, dalloc(c, &k1, (size_t)nnz)); tmps[1] = k1;
    HIPCHK(c, dalloc(c, &v1, (size_t)nnz)); tmps[2] = v1;
    HIPCHK(c, dalloc(c, &hist, (size_t)hcap)); tmps[3] = hist;
    HIPCHK(c, dalloc(c, &stmp, (size_t)scap)); tmps[4] = stmp;

    for (int n = 0; n < N; ++n) {
        auto &md = c->m[n];
        md.I = c->dims[n];
        HIPCHK(c, dalloc(c, &md.perm, (size_t)nnz));
        HIPCHK(c, dalloc(c, &md.rowptr, (size_t)md.I + 1));
        HIPCHK(c, stable_sort_by_key(c->idx, N, n, nnz, key_bits_for(md.I), md.perm, k0, k1, v1,
                                     hist, hcap, stmp, scap, st));
        HIPCHK(c, rowptr_from_sorted(k0, nnz, md.I, md.rowptr, st));
        int t = 0;
        for (int l = 0; l < N; ++l) {
            if (l == n) continue;
            HIPCHK(c, dalloc(c, &md.oidx[t], (size_t)nnz));
            HIPCHK(c, gather_other_index(c->idx, N, l, md.perm, nnz, md.oidx[t], st));
            ++t;
        }
        std::vector<int32_t> rp32((size_t)md.I + 1);
        HIPCHK(c, hipMemcpyAsync(rp32.data(), md.rowptr, rp32.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        md.h_rowptr.assign(rp32.begin(), rp32.end());
        tf_status s = apply_plan(c, n, c->opt.lane_nnz, c->opt.split_threshold, c->opt.chunk_nnz);
        if (s != TF_OK) return s;
        md.persistent = c->opt.strategy == TF_STRATEGY_PERSISTENT;
    }

    // factors (Section 3.1: A^(1) = 0, the others random, so that R = X)
    const size_t sf = ts_size(c->prec);
    uint64_t offset = 0;
    for (int n = 0; n < N; ++n) {
        auto &md = c->m[n];
        HIPCHK(c, ctx_alloc(c, &md.A, (size_t)md.I * c->K * sf));
        const bool zero = c->opt.first_factor_zero && n == 0;
        HIPCHK(c, init_factor(c->prec, md.A, md.I, c->K, c->opt.seed, offset, zero, st));
        offset += (uint64_t)md.I * (uint64_t)c->K;
        const size_t slab = (size_t)md.I * kSlabRowBytes;
        HIPCHK(c, ctx_alloc(c, &md.Z, slab));
        HIPCHK(c, hipMemsetAsync(md.Z, 0, slab, st));
        HIPCHK(c, ctx_alloc(c, &md.rhat, (size_t)nnz * tr_size(c->prec)));
    }
    // residual r = x - reconstruction (exactly x when A^(1) = 0)
    double *r = nullptr;
    HIPCHK(c, dalloc(c, &r, (size_t)nnz));
    const void *A[kMaxModes];
    for (int n = 0; n < N; ++n) A[n] = c->m[n].A;
    hipError_t e = residual_input_order(c->prec, c->idx, c->x, nnz, N, A, c->K,
                                        c->opt.first_factor_zero != 0, r, st);
    for (int n = 0; n < N && e == hipSuccess; ++n)
        e = gather_residual(c->prec, r, c->m[n].perm, nnz, c->m[n].rhat, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(c, r);
    if (e != hipSuccess) return CTX_FAIL(c, TF_E_DEVICE, "residual: %s", hipGetErrorString(e));
    c->order.resize(c->K);
    for (int k = 0; k < c->K; ++k) c->order[k] = k;
    c->pend.clear();
    return TF_OK;
}

}  // namespace

extern "C" {

void tf_default_options(tf_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->size = sizeof(tf_options);
    opt->precision = TF_PREC_F32;
    opt->reg_mode = 0;
    opt->first_factor_zero = 1;
    opt->strategy = TF_STRATEGY_SKEW;
    opt->seed = 2;
    opt->stream = nullptr;
    opt->lane_nnz = 2;
    opt->split_threshold = 4096;
    opt->chunk_nnz = 2048;
    opt->resid_share = TF_RESID_AUTO;
    opt->col_order = TF_ORDER_FIXED;
    opt->mem_budget = 0;
    opt->dev_alloc = nullptr;
    opt->dev_free = nullptr;
    opt->alloc_user = nullptr;
    opt->graph = 0;
}

const char *tf_last_error(const tf_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

tf_status tf_init(tf_ctx **out, int32_t N, const int64_t *dims, int64_t nnz, const int32_t *d_idx,
                  const double *d_vals, int32_t K, double lambda, const tf_options *opt)
{
    g_init_err.clear();
    if (!out) return set_err(&g_init_err, TF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (N < 2 || N > kMaxModes) return set_err(&g_init_err, TF_E_INVALID, "N = %d outside [2, 8]", N);
    if (!dims || !d_idx || !d_vals) return set_err(&g_init_err, TF_E_INVALID, "NULL pointer argument");
    for (int n = 0; n < N; ++n)
        if (dims[n] < 1 || dims[n] > INT32_MAX)
            return set_err(&g_init_err, TF_E_INVALID, "dims[%d] = %lld outside [1, 2^31-1]", n, (long long)dims[n]);
    if (nnz < 1 || nnz > INT32_MAX)
        return set_err(&g_init_err, TF_E_INVALID, "nnz = %lld outside [1, 2^31-1]", (long long)nnz);
    if (K < 1) return set_err(&g_init_err, TF_E_INVALID, "K = %d < 1", K);
    if (!(lambda > 0.0) || !std::isfinite(lambda))
        return set_err(&g_init_err, TF_E_INVALID, "lambda must be positive and finite");
    tf_options o;
    tf_default_options(&o);
    if (opt) {
        if (opt->size != sizeof(tf_options))
            return set_err(&g_init_err, TF_E_INVALID, "tf_options.size mismatch");
        o = *opt;
    }
    if (o.precision < 0 || o.precision > 2) return set_err(&g_init_err, TF_E_INVALID, "bad precision");
    if (o.reg_mode != 0 && o.reg_mode != 1) return set_err(&g_init_err, TF_E_INVALID, "bad reg_mode");
    if (o.strategy != TF_STRATEGY_PLAIN && o.strategy != TF_STRATEGY_SKEW && o.strategy != TF_STRATEGY_AUTO &&
        o.strategy != TF_STRATEGY_PERSISTENT)
        return set_err(&g_init_err, TF_E_INVALID, "bad strategy");
    if (o.col_order != TF_ORDER_FIXED && o.col_order != TF_ORDER_RANDOM)
        return set_err(&g_init_err, TF_E_INVALID, "bad col_order");
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr))
        return set_err(&g_init_err, TF_E_INVALID, "dev_alloc and dev_free must be set together");
    if (o.lane_nnz < 0 || o.split_threshold < 0 || o.chunk_nnz < 0)
        return set_err(&g_init_err, TF_E_INVALID, "negative tuning option");
    if (o.graph != 0 && o.graph != 1) return set_err(&g_init_err, TF_E_INVALID, "bad graph");
    if (o.resid_share < TF_RESID_AUTO || o.resid_share > TF_RESID_SHARED)
        return set_err(&g_init_err, TF_E_INVALID, "bad resid_share");
    if (o.lane_nnz == 0) o.lane_nnz = 2;
    if (o.split_threshold == 0) o.split_threshold = 4096;
    if (o.chunk_nnz == 0) o.chunk_nnz = 2048;

    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return set_err(&g_init_err, TF_E_DEVICE, "no HIP device: %s", hipGetErrorString(he));
    // the device address of tf_foldin_noalloc's scratch array, once per device
    he = fold_scratch_setup(dev);
    if (he != hipSuccess)
        return set_err(&g_init_err, TF_E_DEVICE, "fold-in scratch lookup: %s", hipGetErrorString(he));

    tf_ctx *c = new (std::nothrow) tf_ctx();
    if (!c) return set_err(&g_init_err, TF_E_NOMEM, "host allocation failed");
    c->N = N;
    c->nnz = nnz;
    c->K = K;
    c->lambda = lambda;
    c->opt = o;
    c->prec = o.precision;
    c->stream = (hipStream_t)o.stream;
    if (o.graph && !c->stream) {
        // graphs are captured on a stream of the context's own (a blocking
        // stream at the default priority: ordered with the null stream)
        if (hipStreamCreate(&c->own_stream) != hipSuccess) {
            delete c;
            return set_err(&g_init_err, TF_E_DEVICE, "stream creation failed");
        }
        c->stream = c->own_stream;
    }
    c->device = dev;
    c->err.reserve(512);   // messages up to this length are set without allocating
    for (int n = 0; n < N; ++n) c->dims[n] = dims[n];
    tf_status s = build_state(c, d_idx, d_vals);
    if (s != TF_OK) {
        g_init_err = c->err;
        destroy_ctx(c);
        return s;
    }
    *out = c;
    return TF_OK;
}

void tf_destroy(tf_ctx *ctx) { destroy_ctx(ctx); }

namespace {

// SplitMix64 as a counter-based generator (the factor initialisation's):
// output t for seed s is mix(s + t * 0x9E3779B97F4A7C15).
uint64_t host_splitmix64(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The column permutation of sweep t under TF_ORDER_RANDOM: Fisher-Yates from
// the last position down, position i swapped with j = floor(u (i+1) / 2^53),
// u the top 53 bits of output 2^62 + t K + i.
void draw_col_order(uint64_t seed, int64_t t, int K, std::vector<int32_t> &order)
{
    order.resize(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    for (int i = K - 1; i >= 1; --i) {
        const uint64_t ctr = (1ull << 62) + (uint64_t)t * (uint64_t)K + (uint64_t)i;
        const uint64_t u = host_splitmix64(seed, ctr) >> 11;
        const int j = (int)(((unsigned __int128)u * (unsigned)(i + 1)) >> 53);
        std::swap(order[i], order[j]);
    }
}

// TF_STRATEGY_AUTO: tune each mode's row tiles for the compute width of C
// the first time a split of that width runs.
tf_status auto_tiles(tf_ctx *c, int C, int T_in)
{
    if (c->opt.strategy != TF_STRATEGY_AUTO) return TF_OK;
    const int cp = pick_cp(C, c->prec);
    if (cp < 0 || cp == c->auto_cp) return TF_OK;
    tf_tune_result r;
    const int32_t cand = C;
    const int keep = c->tuned_C;
    tf_status s = tf_autotune(c, T_in, &cand, 1, 1, &r);
    c->tuned_C = keep;
    if (s == TF_OK) c->auto_cp = cp;
    return s;
}

}  // namespace

tf_status tf_split(tf_ctx *ctx, int32_t ncols, const int32_t *h_cols, int32_t T_in)
{
    if (!ctx) return TF_E_INVALID;
    if (!h_cols || ncols < 1 || ncols > ctx->K || T_in < 1)
        return CTX_FAIL(ctx, TF_E_INVALID, "need 1 <= ncols <= K, T_in >= 1");
    for (int q = 0; q < ncols; ++q) {
        if (h_cols[q] < 0 || h_cols[q] >= ctx->K) return CTX_FAIL(ctx, TF_E_INVALID, "column %d out of range", h_cols[q]);
        for (int p = 0; p < q; ++p)
            if (h_cols[p] == h_cols[q]) return CTX_FAIL(ctx, TF_E_INVALID, "column %d repeated", h_cols[q]);
    }
    if (ncols > kMaxBigC) return CTX_FAIL(ctx, TF_E_UNSUPPORTED, "C = %d exceeds %d", ncols, kMaxBigC);
    tf_status s = check_ready(ctx);
    if (s != TF_OK) return s;
    if ((s = auto_tiles(ctx, ncols, T_in)) != TF_OK) return s;
    if ((s = reset_bad(ctx)) != TF_OK) return s;
    if ((s = run_split(ctx, h_cols, ncols, T_in)) != TF_OK) return s;
    return check_bad(ctx);
}

namespace {

// What a sweep's device work depends on besides device data: the sizes,
// flags, plans and buffers its host logic reads.  Equal signatures give the
// same sequence of launches and copies with the same arguments.  (The slab
// geometry is not part of it: every split sets it from its own widths
// before using it, whatever a call between sweeps left.)
std::vector<int64_t> sweep_signature(const tf_ctx *c, int C, int T_in)
{
    auto p = [](const void *q) { return (int64_t)reinterpret_cast<uintptr_t>(q); };
    std::vector<int64_t> v = {C, T_in, (int64_t)c->pend.size(), c->prec, c->K, c->N, c->slab_cp,
                              c->gpart_chunks, p(c->gram), p(c->gpart), p(c->d_cols),
                              p(c->h_ring), c->ring_slots, p(c->d_bad), p(c->stream),
                              c->opt.strategy, c->opt.reg_mode, c->opt.resid_share};
    for (int n = 0; n < c->N; ++n) {
        const auto &md = c->m[n];
        v.insert(v.end(), {md.shared, md.fresh, md.persistent, md.ntasks, p(md.tasks), p(md.items),
                           p(md.chunks), md.nsplit, p(md.split_rows), p(md.split_chunk_ptr),
                           p(md.pos0), p(md.Z), p(md.rhat), p(md.A), md.lane_nnz, md.split_threshold,
                           md.chunk_nnz});
    }
    return v;
}

void save_flags(const tf_ctx *c, std::vector<char> *f)
{
    f->clear();
    for (int n = 0; n < c->N; ++n) {
        f->push_back(c->m[n].shared ? 1 : 0);
        f->push_back(c->m[n].fresh ? 1 : 0);
    }
}

void load_flags(tf_ctx *c, const std::vector<char> &f)
{
    for (int n = 0; n < c->N; ++n) {
        c->m[n].shared = f[2 * n] != 0;
        c->m[n].fresh = f[2 * n + 1] != 0;
    }
}

const int32_t *src_ptr(const tf_ctx *c, const tf_ctx::ColSrc &s, const std::vector<int32_t> &start)
{
    return s.kind == 1 ? c->order.data() + s.begin : s.kind == 2 ? start.data() + s.begin : nullptr;
}

tf_status eager_splits(tf_ctx *c, int C, int T_in)
{
    for (int b = 0; b < c->K; b += C) {
        const int w = std::min(C, c->K - b);
        tf_status s = run_split(c, c->order.data() + b, w, T_in);
        if (s != TF_OK) return s;
    }
    return TF_OK;
}

// Replay of the captured sweep: its column slots rewritten from the current
// order and starting pending list, one graph launch, and the host state the
// captured sweep ended with.
tf_status replay_sweep(tf_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));   // no copy still reads a slot
    const std::vector<int32_t> start = c->pend;
    const size_t slot = 2 * (size_t)c->K + 2;
    for (size_t i = 0; i < c->recipe.size(); ++i) {
        const auto &u = c->recipe[i];
        fill_slot(c, c->h_ring + i * slot, src_ptr(c, u.cur, start), u.cur.len,
                  src_ptr(c, u.pend, start), u.pend.len);
    }
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    const auto &e = c->graph_end_pend;
    const int32_t *ep = src_ptr(c, e, start);
    c->pend.assign(ep, ep + e.len);
    c->pend_src = e;
    load_flags(c, c->graph_end_flags);
    c->ld = c->graph_end_ld;
    c->sw = c->graph_end_sw;
    c->ring_next = (int)c->recipe.size();
    return TF_OK;
}

// The sweep recorded into a graph (nothing runs while recording), then
// launched.  Returns TF_E_STATE with the host state restored when the
// sweep could not be captured; the caller then runs it eagerly.
tf_status capture_sweep(tf_ctx *c, int C, int T_in, const std::vector<int64_t> &sig)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));   // every slot is free again
    const std::vector<int32_t> pend0 = c->pend;
    const tf_ctx::ColSrc src0 = c->pend_src;
    std::vector<char> flags0;
    save_flags(c, &flags0);
    const int ring0 = c->ring_next;
    c->ring_next = 0;
    c->recipe.clear();
    c->pend_src = tf_ctx::ColSrc{pend0.empty() ? 0 : 2, 0, (int)pend0.size()};
    c->capture_bad = false;
    hipGraph_t g = nullptr;
    std::string why;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    tf_status s = TF_E_STATE;
    if (e != hipSuccess) {
        why = std::string("begin: ") + hipGetErrorString(e);
    } else {
        c->capturing = true;
        s = eager_splits(c, C, T_in);
        c->capturing = false;
        if (s != TF_OK) why = "recording: " + c->err;
        e = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess && why.empty()) why = std::string("end: ") + hipGetErrorString(e);
    }
    if (why.empty() && c->capture_bad) why = "a column list not taken from the order";
    hipGraphExec_t x = nullptr;
    if (why.empty() && g) {
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) why = std::string("instantiate: ") + hipGetErrorString(e);
    }
    if (g) (void)hipGraphDestroy(g);
    if (!why.empty() || !x) {
        if (x) (void)hipGraphExecDestroy(x);
        (void)hipGetLastError();
        c->pend = pend0;
        c->pend_src = src0;
        load_flags(c, flags0);
        c->ring_next = ring0;
        // kept for tf_last_error: the sweep itself then runs eagerly
        c->err = "sweep graph not captured (" + why + "); the sweep ran without it";
        return TF_E_STATE;
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = x;
    c->graph_sig = sig;
    c->graph_end_pend = c->pend_src;
    save_flags(c, &c->graph_end_flags);
    c->graph_end_ld = c->ld;
    c->graph_end_sw = c->sw;
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    return TF_OK;
}

}  // namespace

tf_status tf_sweep(tf_ctx *ctx, int32_t C, int32_t T_in)
{
    if (!ctx) return TF_E_INVALID;
    if (C == 0) {
        if (ctx->tuned_C == 0) return CTX_FAIL(ctx, TF_E_STATE, "C = 0 needs tf_autotune first");
        C = ctx->tuned_C;
    }
    if (C < 1 || C > ctx->K || T_in < 1) return CTX_FAIL(ctx, TF_E_INVALID, "need 1 <= C <= K, T_in >= 1");
    if (C > kMaxBigC) return CTX_FAIL(ctx, TF_E_UNSUPPORTED, "C = %d exceeds %d", C, kMaxBigC);
    tf_status s = check_ready(ctx);
    if (s != TF_OK) return s;
    if ((s = auto_tiles(ctx, C, T_in)) != TF_OK) return s;
    if ((s = reset_bad(ctx)) != TF_OK) return s;
    if (ctx->opt.col_order == TF_ORDER_RANDOM) draw_col_order(ctx->opt.seed, ctx->sweeps_run, ctx->K, ctx->order);
    ctx->sweeps_run += 1;
    // A graph holds the narrow and 32-column paths (no workgroup-per-row
    // splits, no profiling events); it is recorded the second time a
    // starting state is seen, when every lazy allocation has been made.
    const int nsplit = (ctx->K + C - 1) / C;
    bool graphed = false;
    if (ctx->opt.graph && !ctx->profiling &&
        pick_cp(std::max<int>(C, (int)ctx->pend.size()), ctx->prec) > 0) {
        if ((s = ensure_ring(ctx, 2 * nsplit + 2)) != TF_OK) return s;
        const std::vector<int64_t> sig = sweep_signature(ctx, C, T_in);
        if (ctx->graph_exec && sig == ctx->graph_sig) {
            if ((s = replay_sweep(ctx)) != TF_OK) return s;
            graphed = true;
        } else if (sig == ctx->last_sig) {
            s = capture_sweep(ctx, C, T_in, sig);
            if (s == TF_OK) graphed = true;
            else if (s != TF_E_STATE) return s;
        }
        ctx->last_sig = sig;
    }
    if (!graphed && (s = eager_splits(ctx, C, T_in)) != TF_OK) return s;
    ctx->kstats.sweeps += 1;
    if (graphed) ctx->kstats.graph_sweeps += 1;
    return check_bad(ctx);
}

namespace {

// One timed pass on mode n (accumulation, chunk sums, solve) reading the
// residual from `rhat` (through `rperm` when given: a plain pass on mode
// 0's copy); returns milliseconds.
tf_status time_pass(tf_ctx *c, int n, int CP, int npend, bool first, void *rhat, double *ms,
                    const int32_t *rperm = nullptr)
{
    auto &md = c->m[n];
    AccumArgs a;
    fill_accum_args(c, n, first ? npend : 0, &a);
    a.rhat = rhat;
    a.rperm = rperm;
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return CTX_FAIL(c, TF_E_DEVICE, "event creation failed");
    HIPCHK(c, hipEventRecord(e0, c->stream));
    const int grid = (md.ntasks + 3) / 4;
    if (grid > 0) {
        tf_status s0 = reset_work(c, a);
        if (s0 != TF_OK) return s0;
        HIPCHK(c, launch_accum(c->prec, CP, c->N - 1, first, a, grid, c->stream));
    }
    if (md.nsplit > 0)
        HIPCHK(c, launch_chunk_reduce(c->prec, CP, md.split_rows, md.split_chunk_ptr, md.nsplit,
                                      c->gpart, c->gram, c->stream));
    SolveArgs sa;
    sa.rowptr = md.rowptr; sa.I = md.I; sa.gram = c->gram; sa.W = md.Z; sa.ld = c->ld;
    sa.lambda = c->lambda; sa.reg_mode = c->opt.reg_mode; sa.bad = c->d_bad + n;
    sa.flags = c->d_bad; sa.nmodes = c->N;
    HIPCHK(c, launch_solve(c->prec, CP, sa, c->stream));
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(c, hipEventElapsedTime(&f, e0, e1));
    c->ev_free.push_back(e0);
    c->ev_free.push_back(e1);
    *ms = f;
    return TF_OK;
}

// Set up a steady-state trial split of width C: current columns order[0..C),
// pending columns the last C of the order, slabs packed for both.
tf_status trial_slabs(tf_ctx *c, int C, int *CP_out, int *npend_out)
{
    const int CP = pick_cp(C, c->prec);
    if (CP < 0) return CTX_FAIL(c, TF_E_UNSUPPORTED, "C = %d not runnable in this precision", C);
    tf_status s = ensure_gram(c, CP);
    if (s != TF_OK) return s;
    const int npend = C;
    std::vector<int32_t> cols(c->order.begin(), c->order.begin() + C);
    const auto saved = c->pend;
    c->pend.assign(c->order.end() - C, c->order.end());
    s = slab_geometry(c, CP);
    if (s == TF_OK) s = upload_cols(c, cols.data(), C);
    c->pend = saved;
    if (s != TF_OK) return s;
    if ((s = pack_all(c, c->d_cols, C, c->d_cols + c->K, npend)) != TF_OK) return s;
    *CP_out = CP;
    *npend_out = npend;
    return TF_OK;
}

// Times of mode n's first and later passes in a trial split, with the
// residual placement a real split of this width would use; own-copy passes
// work on a scratch copy of the residual.
tf_status time_mode(tf_ctx *c, int n, int CP, int npend, int T_in, void *scratch, double *t1,
                    double *t2)
{
    tf_status s;
    *t1 = *t2 = 0.0;
    if (want_shared(c, n, CP, npend, T_in)) {
        if ((s = ensure_pos0(c, n)) != TF_OK) return s;
        if ((s = time_pass(c, n, CP, 0, false, c->m[0].rhat, t1, c->m[n].pos0)) != TF_OK) return s;
        *t2 = *t1;
        return TF_OK;
    }
    if (!c->m[n].fresh) {
        HIPCHK(c, gather_copy(c->prec, c->m[0].rhat, c->m[n].pos0, c->nnz, scratch, c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(scratch, c->m[n].rhat, (size_t)c->nnz * tr_size(c->prec),
                                 hipMemcpyDeviceToDevice, c->stream));
    }
    if ((s = time_pass(c, n, CP, npend, true, scratch, t1)) != TF_OK) return s;
    if (T_in > 1 && (s = time_pass(c, n, CP, npend, false, scratch, t2)) != TF_OK) return s;
    return TF_OK;
}

// Mode n's pass time for the tiles being tried: the shorter of two trials
// (one trial's noise, a few percent, is as large as the differences between
// neighbouring tiles).
tf_status time_mode_best(tf_ctx *c, int n, int C, int T_in, void *scratch, double *t)
{
    *t = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        int CP = 0, npend = 0;
        tf_status s = trial_slabs(c, C, &CP, &npend);
        if (s != TF_OK) return s;
        double t1 = 0.0, t2 = 0.0;
        if ((s = time_mode(c, n, CP, npend, T_in, scratch, &t1, &t2)) != TF_OK) return s;
        *t = std::min(*t, t1 + (T_in - 1) * t2);
    }
    return TF_OK;
}

}  // namespace

extern "C" tf_status tf_autotune(tf_ctx *ctx, int32_t T_in, const int32_t *h_cands, int32_t ncand,
                                 int32_t tune_tiles, tf_tune_result *out)
{
    if (!ctx) return TF_E_INVALID;
    if (!h_cands || ncand < 1 || ncand > 16 || T_in < 1 || !out)
        return CTX_FAIL(ctx, TF_E_INVALID, "need 1..16 candidates, T_in >= 1, an output");
    for (int q = 0; q < ncand; ++q)
        if (h_cands[q] < 1 || h_cands[q] > ctx->K || pick_cp(h_cands[q], ctx->prec) < 0)
            return CTX_FAIL(ctx, TF_E_INVALID, "candidate C = %d not runnable", h_cands[q]);
    tf_status s = check_ready(ctx);
    if (s != TF_OK) return s;
    const auto t_start = std::chrono::steady_clock::now();
    std::memset(out, 0, sizeof *out);
    void *scratch = nullptr;
    HIPCHK(ctx, ctx_alloc(ctx, &scratch, (size_t)ctx->nnz * tr_size(ctx->prec)));
    struct Free { tf_ctx *c; void *p; ~Free() { dfree(c, p); } } guard{ctx, scratch};
    if ((s = reset_bad(ctx)) != TF_OK) return s;

    double best = 1e300;
    int bestC = h_cands[0];
    for (int q = 0; q < ncand; ++q) {
        const int C = h_cands[q];
        int CP = 0, npend = 0;
        if ((s = trial_slabs(ctx, C, &CP, &npend)) != TF_OK) return s;
        double split_ms = 0.0;
        for (int n = 0; n < ctx->N; ++n) {
            double t1 = 0.0, t2 = 0.0;
            if ((s = time_mode(ctx, n, CP, npend, T_in, scratch, &t1, &t2)) != TF_OK) return s;
            split_ms += t1 + (T_in - 1) * t2;
        }
        // slab packing and write-back: time one packing of all modes, count it twice
        hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx);
        HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
        if ((s = pack_all(ctx, ctx->d_cols, C, ctx->d_cols + ctx->K, npend)) != TF_OK) return s;
        HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
        HIPCHK(ctx, hipEventSynchronize(e1));
        float pk = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&pk, e0, e1));
        ctx->ev_free.push_back(e0);
        ctx->ev_free.push_back(e1);
        const double est = (double)((ctx->K + C - 1) / C) * (split_ms + 2.0 * pk);
        out->cand_C[q] = C;
        out->est_sweep_ms[q] = est;
        if (est < best) { best = est; bestC = C; }
    }
    out->ncand = ncand;
    out->best_C = bestC;
    ctx->tuned_C = bestC;

    if (tune_tiles) {
        static const int lanes[] = {1, 2, 4, 8};
        static const int chunks[] = {1024, 4096, 16384};
        for (int n = 0; n < ctx->N; ++n) {
            double tbest = 1e300;
            int bl = ctx->m[n].lane_nnz, bs = ctx->m[n].split_threshold, bc = ctx->m[n].chunk_nnz;
            for (int lane : lanes)
                for (int ch : chunks) {
                    if ((s = apply_plan(ctx, n, lane, 2 * ch, ch)) != TF_OK) return s;
                    double t = 0.0;
                    if ((s = time_mode_best(ctx, n, bestC, T_in, scratch, &t)) != TF_OK) return s;
                    if (t < tbest) { tbest = t; bl = lane; bs = 2 * ch; bc = ch; }
                }
            if ((s = apply_plan(ctx, n, bl, bs, bc)) != TF_OK) return s;
            // the launch form for these tiles (unless the caller fixed it):
            // a grid of one wavefront per task, or one resident grid whose
            // wavefronts take tasks from a counter (same results bit for bit)
            if (ctx->opt.strategy == TF_STRATEGY_SKEW || ctx->opt.strategy == TF_STRATEGY_AUTO) {
                double tf_[2];
                for (int p = 0; p < 2; ++p) {
                    ctx->m[n].persistent = p == 1;
                    if ((s = time_mode_best(ctx, n, bestC, T_in, scratch, &tf_[p])) != TF_OK) return s;
                }
                ctx->m[n].persistent = tf_[1] < tf_[0];
            }
        }
        if ((s = ensure_gram(ctx, pick_cp(bestC, ctx->prec))) != TF_OK) return s;
    }
    for (int n = 0; n < ctx->N && n < 8; ++n) {
        out->lane_nnz[n] = ctx->m[n].lane_nnz;
        out->split_threshold[n] = ctx->m[n].split_threshold;
        out->chunk_nnz[n] = ctx->m[n].chunk_nnz;
        out->persistent[n] = ctx->m[n].persistent ? 1 : 0;
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    out->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return TF_OK;
}

tf_status tf_set_col_order(tf_ctx *ctx, const int32_t *h_order)
{
    if (!ctx) return TF_E_INVALID;
    if (!h_order) return CTX_FAIL(ctx, TF_E_INVALID, "NULL order");
    std::vector<char> seen(ctx->K, 0);
    for (int k = 0; k < ctx->K; ++k) {
        if (h_order[k] < 0 || h_order[k] >= ctx->K || seen[h_order[k]])
            return CTX_FAIL(ctx, TF_E_INVALID, "order is not a permutation of 0..K-1");
        seen[h_order[k]] = 1;
    }
    ctx->order.assign(h_order, h_order + ctx->K);
    return TF_OK;
}

tf_status tf_get_col_order(const tf_ctx *ctx, int32_t *h_order)
{
    if (!ctx || !h_order) return TF_E_INVALID;
    std::memcpy(h_order, ctx->order.data(), ctx->K * sizeof(int32_t));
    return TF_OK;
}

tf_status tf_loss(tf_ctx *ctx, double *loss, double *train_rmse)
{
    if (!ctx) return TF_E_INVALID;
    tf_status s = check_ready(ctx);
    if (s != TF_OK) return s;
    double se = 0.0;
    if ((s = eval_residual(ctx, nullptr, &se)) != TF_OK) return s;
    int64_t nb_total = 0;
    int nb[kMaxModes];
    for (int n = 0; n < ctx->N; ++n) {
        nb[n] = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (ctx->m[n].I + 255) / 256));
        nb_total += nb[n];
    }
    if ((s = ensure_partials(ctx, nb_total)) != TF_OK) return s;
    int64_t off = 0;
    for (int n = 0; n < ctx->N; ++n) {
        HIPCHK(ctx, reg_partials(ctx->prec, ctx->m[n].A, ctx->m[n].I, ctx->K, ctx->m[n].rowptr,
                                 ctx->opt.reg_mode, ctx->d_partials + off, nb[n], ctx->stream));
        off += nb[n];
    }
    HIPCHK(ctx, sum_partials(ctx->d_partials, nb_total, ctx->d_scalar + 1, ctx->stream));
    double reg = 0.0;
    HIPCHK(ctx, hipMemcpyAsync(&reg, ctx->d_scalar + 1, sizeof reg, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (loss) *loss = se + ctx->lambda * reg;
    if (train_rmse) *train_rmse = std::sqrt(se / (double)ctx->nnz);
    if (!std::isfinite(se) || !std::isfinite(reg))
        return CTX_FAIL(ctx, TF_E_NUMERIC, "loss is not finite");
    return TF_OK;
}

tf_status tf_get_residual(tf_ctx *ctx, double *h)
{
    if (!ctx) return TF_E_INVALID;
    if (!h) return CTX_FAIL(ctx, TF_E_INVALID, "NULL output");
    tf_status s = check_ready(ctx);
    if (s != TF_OK) return s;
    double *d = nullptr;
    HIPCHK(ctx, dalloc(ctx, &d, (size_t)ctx->nnz));
    double se = 0.0;
    s = eval_residual(ctx, d, &se);
    if (s == TF_OK) {
        hipError_t e = hipMemcpy(h, d, (size_t)ctx->nnz * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) s = CTX_FAIL(ctx, TF_E_DEVICE, "copy: %s", hipGetErrorString(e));
    }
    dfree(ctx, d);
    return s;
}

tf_status tf_resync(tf_ctx *ctx)
{
    if (!ctx) return TF_E_INVALID;
    double *r = nullptr;
    HIPCHK(ctx, dalloc(ctx, &r, (size_t)ctx->nnz));
    const void *A[kMaxModes];
    for (int n = 0; n < ctx->N; ++n) A[n] = ctx->m[n].A;
    hipError_t e = residual_input_order(ctx->prec, ctx->idx, ctx->x, ctx->nnz, ctx->N, A, ctx->K,
                                        false, r, ctx->stream);
    for (int n = 0; n < ctx->N && e == hipSuccess; ++n)
        e = gather_residual(ctx->prec, r, ctx->m[n].perm, ctx->nnz, ctx->m[n].rhat, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dfree(ctx, r);
    if (e != hipSuccess) return CTX_FAIL(ctx, TF_E_DEVICE, "resync: %s", hipGetErrorString(e));
    for (int n = 0; n < ctx->N; ++n) ctx->m[n].fresh = true;
    ctx->pend.clear();
    ctx->stale = false;
    return TF_OK;
}

tf_status tf_get_factor(tf_ctx *ctx, int32_t n, double *h)
{
    if (!ctx) return TF_E_INVALID;
    if (n < 0 || n >= ctx->N || !h) return CTX_FAIL(ctx, TF_E_INVALID, "bad mode or NULL output");
    const int64_t cnt = ctx->m[n].I * ctx->K;
    double *d = nullptr;
    HIPCHK(ctx, dalloc(ctx, &d, (size_t)cnt));
    hipError_t e = factor_to_f64(ctx->prec, ctx->m[n].A, cnt, d, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(h, d, (size_t)cnt * sizeof(double), hipMemcpyDeviceToHost);
    dfree(ctx, d);
    if (e != hipSuccess) return CTX_FAIL(ctx, TF_E_DEVICE, "get_factor: %s", hipGetErrorString(e));
    return TF_OK;
}

tf_status tf_get_factor_block(tf_ctx *ctx, int32_t n, int64_t nrows, const int32_t *h_rows,
                             int32_t ncols, const int32_t *h_cols, double *h)
{
    if (!ctx) return TF_E_INVALID;
    if (n < 0 || n >= ctx->N || !h) return CTX_FAIL(ctx, TF_E_INVALID, "bad mode or NULL output");
    const int64_t I = ctx->m[n].I;
    if (h_rows ? (nrows < 1 || nrows > I) : nrows != I)
        return CTX_FAIL(ctx, TF_E_INVALID, "row count %lld does not fit mode %d", (long long)nrows, n);
    if (h_cols ? (ncols < 1 || ncols > ctx->K) : ncols != ctx->K)
        return CTX_FAIL(ctx, TF_E_INVALID, "column count %d does not fit K = %d", ncols, ctx->K);
    if (h_rows)
        for (int64_t q = 0; q < nrows; ++q)
            if (h_rows[q] < 0 || h_rows[q] >= I) return CTX_FAIL(ctx, TF_E_INVALID, "row %d out of range", h_rows[q]);
    if (h_cols)
        for (int q = 0; q < ncols; ++q)
            if (h_cols[q] < 0 || h_cols[q] >= ctx->K) return CTX_FAIL(ctx, TF_E_INVALID, "column %d out of range", h_cols[q]);
    const int64_t cnt = nrows * ncols;
    double *d = nullptr;
    int32_t *dr = nullptr, *dc = nullptr;
    HIPCHK(ctx, dalloc(ctx, &d, (size_t)cnt));
    hipError_t e = hipSuccess;
    if (h_rows) {
        e = dalloc(ctx, &dr, (size_t)nrows);
        if (e == hipSuccess) e = hipMemcpy(dr, h_rows, (size_t)nrows * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && h_cols) {
        e = dalloc(ctx, &dc, (size_t)ncols);
        if (e == hipSuccess) e = hipMemcpy(dc, h_cols, (size_t)ncols * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = factor_block_to_f64(ctx->prec, ctx->m[n].A, ctx->K, dr, nrows, dc, ncols, d, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(h, d, (size_t)cnt * sizeof(double), hipMemcpyDeviceToHost);
    dfree(ctx, d);
    dfree(ctx, dr);
    dfree(ctx, dc);
    if (e != hipSuccess) return CTX_FAIL(ctx, TF_E_DEVICE, "get_factor_block: %s", hipGetErrorString(e));
    return TF_OK;
}

tf_status tf_set_factor(tf_ctx *ctx, int32_t n, const double *h)
{
    if (!ctx) return TF_E_INVALID;
    if (n < 0 || n >= ctx->N || !h) return CTX_FAIL(ctx, TF_E_INVALID, "bad mode or NULL input");
    const int64_t cnt = ctx->m[n].I * ctx->K;
    for (int64_t t = 0; t < cnt; ++t)
        if (!std::isfinite(h[t])) return CTX_FAIL(ctx, TF_E_INVALID, "factor entry %lld is not finite", (long long)t);
    double *d = nullptr;
    HIPCHK(ctx, dalloc(ctx, &d, (size_t)cnt));
    hipError_t e = hipMemcpy(d, h, (size_t)cnt * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = factor_from_f64(ctx->prec, d, cnt, ctx->m[n].A, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dfree(ctx, d);
    if (e != hipSuccess) return CTX_FAIL(ctx, TF_E_DEVICE, "set_factor: %s", hipGetErrorString(e));
    ctx->stale = true;
    return TF_OK;
}

tf_status tf_get_csr(tf_ctx *ctx, int32_t n, int64_t *h_rowptr, int32_t *h_perm)
{
    if (!ctx) return TF_E_INVALID;
    if (n < 0 || n >= ctx->N || !h_rowptr || !h_perm) return CTX_FAIL(ctx, TF_E_INVALID, "bad arguments");
    std::vector<int32_t> rp((size_t)ctx->m[n].I + 1);
    HIPCHK(ctx, hipMemcpy(rp.data(), ctx->m[n].rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < rp.size(); ++i) h_rowptr[i] = rp[i];
    HIPCHK(ctx, hipMemcpy(h_perm, ctx->m[n].perm, (size_t)ctx->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    return TF_OK;
}

tf_status tf_predict(tf_ctx *ctx, int64_t m, const int32_t *d_idx, double *d_out)
{
    if (!ctx) return TF_E_INVALID;
    if (m < 0) return CTX_FAIL(ctx, TF_E_INVALID, "m < 0");
    if (m == 0) return TF_OK;
    if (!d_idx || !d_out) return CTX_FAIL(ctx, TF_E_INVALID, "NULL pointer argument");
    const void *A[kMaxModes];
    for (int n = 0; n < ctx->N; ++n) A[n] = ctx->m[n].A;
    HIPCHK(ctx, hipMemsetAsync(ctx->d_bad, 0xff, sizeof(unsigned long long), ctx->stream));
    HIPCHK(ctx, launch_predict(ctx->prec, ctx->N, ctx->K, A, ctx->dims, d_idx, m, d_out, ctx->d_bad, ctx->stream));
    unsigned long long hb = 0;
    HIPCHK(ctx, hipMemcpyAsync(&hb, ctx->d_bad, sizeof hb, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (hb != ULLONG_MAX) return CTX_FAIL(ctx, TF_E_INVALID, "query %llu has an index out of range", hb);
    return TF_OK;
}

tf_status tf_profile(tf_ctx *ctx, int32_t enable)
{
    if (!ctx) return TF_E_INVALID;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &t : ctx->ev_pending) { ctx->ev_free.push_back(t.a); ctx->ev_free.push_back(t.b); }
    ctx->ev_pending.clear();
    ctx->kstats = tf_kstats{};
    ctx->profiling = enable != 0;
    return TF_OK;
}

tf_status tf_profile_read(tf_ctx *ctx, tf_kstats *out)
{
    if (!ctx || !out) return TF_E_INVALID;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &t : ctx->ev_pending) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->kstats.launches += 1;
        ctx->kstats.total_ms += ms;
        ctx->kstats.alg_bytes += t.bytes;
        if (t.first) {
            ctx->kstats.first_launches += 1;
            ctx->kstats.first_ms += ms;
            ctx->kstats.first_bytes += t.bytes;
        }
        ctx->ev_free.push_back(t.a);
        ctx->ev_free.push_back(t.b);
    }
    ctx->ev_pending.clear();
    *out = ctx->kstats;
    return TF_OK;
}

}  // extern "C"
