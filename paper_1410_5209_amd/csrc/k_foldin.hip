// Fold-in of new rows against resident factors (a use of the row update of
// arXiv:1410.5209 that the paper does not make itself): a request is a new
// row of one mode given by its observed entries (indices of the other modes
// and values).  Full rank solves eq. (ALS) for the row, a = (B + lambda_i I)^-1 c
// with c built from the values; CDTF runs coordinate sweeps of the C = 1
// update starting from a = 0.  Both start from the request's Gram matrix
// B = P^T P and c = P^T x: the entries are cut into fixed chunks (one
// workgroup each, partial records in the accumulation type) summed in chunk
// order in FP64, so a request's result does not depend on the batch it
// travels in.
#include <climits>

#include "dev_common.h"
#include "foldin.h"

namespace tfk {

// P[j][k] = prod over the other modes of the resident factor rows.
template <int PREC>
__global__ void k_fold_p(FoldArgs a, int64_t total)
{
    using TS = typename Types<PREC>::TS;
    using TA = typename Types<PREC>::TA;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total * a.K) return;
    const int64_t j = t / a.K;
    const int k = (int)(t - j * a.K);
    TA p = TA(1);
    int q = 0;
    for (int l = 0; l < a.N; ++l) {
        if (l == a.mode) continue;
        const int32_t i = a.oidx[j * (a.N - 1) + q];
        p *= (TA)load_f64(reinterpret_cast<const TS *>(a.A[l]) + (int64_t)i * a.K + k);
        ++q;
    }
    reinterpret_cast<TA *>(a.P)[t] = p;
}

__global__ void k_fold_validate(FoldArgs a, int64_t total, Dims8x d)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    bool bad = !isfinite(a.vals[j]);
    int q = 0;
    for (int l = 0; l < a.N; ++l) {
        if (l == a.mode) continue;
        const int32_t i = a.oidx[j * (a.N - 1) + q];
        bad = bad || i < 0 || (int64_t)i >= d.d[l];
        ++q;
    }
    if (bad) atomicMin(a.bad, (unsigned long long)j);
}

// Deterministic sums of two values over a 256-thread block (fixed tree).
__device__ __forceinline__ void fold_block_sum2(double &u, double &v, double *scratch)
{
    for (int m = 32; m >= 1; m >>= 1) {
        u += __shfl_xor(u, m, 64);
        v += __shfl_xor(v, m, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        scratch[threadIdx.x >> 6] = u;
        scratch[4 + (threadIdx.x >> 6)] = v;
    }
    __syncthreads();
    u = (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
    v = (scratch[4] + scratch[5]) + (scratch[6] + scratch[7]);
}

constexpr int FOLD_CHUNK = 32;   // entries staged per step
constexpr int FOLD_RB = 8;       // register block per thread (8 x 8 -> K <= 128)

// Partial Gram of one chunk of one request (K <= 128): B and c over the
// chunk's entries in the accumulation type, written as a record of the lower
// triangle of B then c.  Thread (ty, tx) accumulates rows ty + 16u and
// columns tx + 16v of B for the blocks v <= u that reach below row K.  (The
// entries' p rows come from k_fold_p, which forms them across the whole GPU:
// forming them here, chunk by chunk, made this kernel twice as slow.)
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_gram(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    __shared__ double xs[FOLD_CHUNK];
    extern __shared__ double smem[];
    const int K = a.K;
    const int cidx = blockIdx.x;
    const int q = a.chunk_req[cidx];
    const int64_t beg = a.req_ptr[q] + (int64_t)(cidx - a.chunk_first[q]) * kFoldChunkEntries;
    const int64_t end = min(a.req_ptr[q + 1], beg + kFoldChunkEntries);
    const int tid = threadIdx.x;
    TA *Pc = reinterpret_cast<TA *>(smem);
    const int ty = tid >> 4, tx = tid & 15;
    TA acc[FOLD_RB][FOLD_RB];
#pragma unroll
    for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
        for (int v = 0; v < FOLD_RB; ++v) acc[u][v] = TA(0);
    TA racc = TA(0);   // c entry k = tid (tid < K)

    const TA *P = reinterpret_cast<const TA *>(a.P);
    const int nub = (K + 15) / 16;   // row blocks that reach below K
    for (int64_t c0 = beg; c0 < end; c0 += FOLD_CHUNK) {
        const int cn = (int)(end - c0 < FOLD_CHUNK ? end - c0 : FOLD_CHUNK);
        for (int e = tid; e < cn * K; e += 256) Pc[e] = P[c0 * K + e];
        if (tid < cn) xs[tid] = a.vals[c0 + tid];
        __syncthreads();
#pragma unroll 2
        for (int j = 0; j < cn; ++j) {
            TA pr[FOLD_RB], pc[FOLD_RB];
#pragma unroll
            for (int u = 0; u < FOLD_RB; ++u) {
                const int k1 = ty + 16 * u, k2 = tx + 16 * u;
                pr[u] = k1 < K ? Pc[j * K + k1] : TA(0);
                pc[u] = k2 < K ? Pc[j * K + k2] : TA(0);
            }
#pragma unroll
            for (int u = 0; u < FOLD_RB; ++u) {
                if (u >= nub) continue;
#pragma unroll
                for (int v = 0; v <= u; ++v) acc[u][v] += pr[u] * pc[v];
            }
            if (tid < K) racc += (TA)xs[j] * Pc[j * K + tid];
        }
        __syncthreads();
    }
    TA *out = reinterpret_cast<TA *>(a.gpart) + (int64_t)cidx * fold_gram_stride(K);
#pragma unroll
    for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
        for (int v = 0; v <= u; ++v) {
            const int k1 = ty + 16 * u, k2 = tx + 16 * v;
            if (k1 < K && k2 <= k1) out[k1 * (k1 + 1) / 2 + k2] = acc[u][v];
        }
    if (tid < K) out[K * (K + 1) / 2 + tid] = racc;
}

// Elements e0 + u * nb (u < U) of a request's nc chunk records, each summed
// over the chunks in chunk order, CT chunks at a time.  The loads are not
// conditional (indices past the ends are clamped and their values dropped),
// so a group of them is issued together.
template <typename TA, int CT>
__device__ __forceinline__ void sum_records_group(const TA *gp, int64_t gs, int nc, int e0, int nb,
                                                  int total, int KT, double *L, double *rhs)
{
    constexpr int U = 4;
    double sum[U];
    int eu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        sum[u] = 0.0;
        const int e = e0 + u * nb;
        eu[u] = e < total ? e : total - 1;
    }
    for (int t0 = 0; t0 < nc; t0 += CT) {
        TA v[CT][U];
#pragma unroll
        for (int tt = 0; tt < CT; ++tt) {
            const int64_t row = (int64_t)(t0 + tt < nc ? t0 + tt : nc - 1) * gs;
#pragma unroll
            for (int u = 0; u < U; ++u) v[tt][u] = gp[row + eu[u]];
        }
#pragma unroll
        for (int tt = 0; tt < CT; ++tt)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t0 + tt < nc) sum[u] += (double)v[tt][u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = e0 + u * nb;
        if (e >= total) continue;
        if (e < KT) L[e] = sum[u];
        else rhs[e - KT] = sum[u];
    }
}

// A request's Gram record (packed lower triangle of B, then c): the sum of
// its chunk records in chunk order, in FP64; the chunk group matches the
// request's size (most requests have one chunk).
template <typename TA>
__device__ __forceinline__ void sum_chunk_records(const FoldArgs &a, int q, double *L, double *rhs)
{
    const int K = a.K;
    const int KT = K * (K + 1) / 2;
    const int64_t gs = fold_gram_stride(K);
    const int c0 = a.chunk_first[q], nc = a.chunk_first[q + 1] - c0;
    const TA *gp = reinterpret_cast<const TA *>(a.gpart) + (int64_t)c0 * gs;
    const int nb = blockDim.x, total = KT + K;
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * nb) {
        if (nc == 1) sum_records_group<TA, 1>(gp, gs, nc, e0, nb, total, KT, L, rhs);
        else if (nc <= 4) sum_records_group<TA, 4>(gp, gs, nc, e0, nb, total, KT, L, rhs);
        else sum_records_group<TA, 16>(gp, gs, nc, e0, nb, total, KT, L, rhs);
    }
}

// Packed lower triangle: element (i, k), k <= i.
__device__ __forceinline__ int tri(int i, int k) { return i * (i + 1) / 2 + k; }

// A double held by lane j, to every lane of the wavefront.
__device__ __forceinline__ double lane_bcast(double v, int j)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
    return __hiloint2double(hi, lo);
}

// Sum over the wavefront, the same in every lane, in a fixed order: DPP
// steps within each row of 16 lanes, then the four row sums by lane reads.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_mov<0xB1>(v);    // quad_perm 1,0,3,2
    v += dpp_mov<0x4E>(v);    // quad_perm 2,3,0,1
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

constexpr int kPanel = 32;   // columns per panel of the blocked Cholesky

// 1 / sqrt(d) for d > 0: the hardware estimate and two steps of Newton's
// iteration r <- r (3 - d r^2) / 2, each roughly doubling the correct bits.
__device__ __forceinline__ double fold_rsqrt(double d)
{
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}

// Cholesky of the diagonal block (rows and columns c0 .. c0 + w - 1, w <=
// 32) of the packed triangle, in place, by one wavefront: lane i holds row i
// of the block in registers.  Step j: lane j's pivot reaches every lane by
// lane reads; lanes i > j form L(i, j) and publish it in col[]; every lane
// updates its row from there (LDS accesses of one wavefront stay in program
// order).  rdiag[c0 + j] = 1 / L(j, j).  A non-positive pivot sets *failed
// and the factorisation goes on with 1 (the request is then reported).
__device__ __forceinline__ void fold_diag_block(double *L, int c0, int w, double *rdiag, double *col, int *failed)
{
    const int i = threadIdx.x & 63;
    const bool in = i < w;
    double m[kPanel];
#pragma unroll
    for (int k = 0; k < kPanel; ++k) m[k] = (in && k <= i) ? L[tri(c0 + i, c0 + k)] : 0.0;
#pragma unroll
    for (int j = 0; j < kPanel; ++j) {
        if (j >= w) continue;   // (not break: the loop must unroll fully)
        const double d = lane_bcast(m[j], j);
        const bool ok = d > 0.0;
        const double dd = ok ? d : 1.0, rinv = fold_rsqrt(dd), ljj = dd * rinv;
        if (i == 0 && !ok) *failed = 1;
        double lij = 0.0;
        if (in && i > j) {
            lij = m[j] * rinv;
            m[j] = lij;
            col[i] = lij;
        }
        if (i == j) {
            m[j] = ljj;
            rdiag[c0 + j] = rinv;
        }
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
        // M(i, k) -= L(i, j) L(k, j) for k > j (lanes with no row, or k
        // beyond their row, update scratch registers that are not stored)
#pragma unroll
        for (int k = j + 1; k < kPanel; ++k) m[k] -= lij * col[k];
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int k = 0; k < kPanel; ++k)
        if (in && k <= i) L[tri(c0 + i, c0 + k)] = m[k];
}

// Rows below the diagonal block: L(r, c0..) = A(r, c0..) L11^{-T}, one
// thread per row, forward substitution against the block.
__device__ __forceinline__ void fold_panel_rows(double *L, int c0, int w, int K, const double *rdiag)
{
    for (int r = c0 + w + (int)threadIdx.x; r < K; r += blockDim.x) {
        const int base = tri(r, c0);
        double x[kPanel];
#pragma unroll
        for (int k = 0; k < kPanel; ++k) x[k] = k < w ? L[base + k] : 0.0;
#pragma unroll
        for (int k = 0; k < kPanel; ++k) {
            if (k >= w) continue;
            double s = x[k];
            const int bk = tri(c0 + k, c0);
#pragma unroll
            for (int t = 0; t < k; ++t) s -= x[t] * L[bk + t];
            x[k] = s * rdiag[c0 + k];
        }
#pragma unroll
        for (int k = 0; k < kPanel; ++k)
            if (k < w) L[base + k] = x[k];
    }
}

// Trailing update of the rows and columns after the panel, in 4 x 4 tiles
// of the lower triangle: A(r, s) -= sum_k L(r, k) L(s, k) over the panel.
__device__ __forceinline__ void fold_trailing(double *L, int c0, int w, int K)
{
    const int c1 = c0 + w, n = K - c1;
    if (n <= 0) return;
    const int T = (n + 3) / 4, ntile = T * (T + 1) / 2;
    for (int t = threadIdx.x; t < ntile; t += blockDim.x) {
        int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        const int tj = t - ti * (ti + 1) / 2;
        const int r0 = c1 + 4 * ti, s0 = c1 + 4 * tj;
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
        for (int k = 0; k < w; ++k) {
            double ra[4], sb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ra[u] = r0 + u < K ? L[tri(r0 + u, c0 + k)] : 0.0;
                sb[u] = s0 + u < K ? L[tri(s0 + u, c0 + k)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += ra[u] * sb[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + u, c = s0 + v;
                if (r < K && c <= r) L[tri(r, c)] -= acc[u][v];
            }
    }
}

// Full-rank fold-in of one request per workgroup (K <= 128): the chunk
// records summed in chunk order in FP64, then eq. (ALS) by Cholesky.
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_full(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    extern __shared__ double smem[];
    const int K = a.K;
    const int q = blockIdx.x;
    const int64_t beg = a.req_ptr[q], end = a.req_ptr[q + 1];
    const int64_t m = end - beg;
    double *out = a.rows + (int64_t)q * K;
    const int tid = threadIdx.x;
    if (m == 0) {
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        if (tid == 0 && a.req_status) a.req_status[q] = TF_OK;
        return;
    }
    // LDS: packed lower triangle L (K(K+1)/2 doubles), rhs (K doubles)
    double *L = smem;
    double *rhs = L + K * (K + 1) / 2;
    sum_chunk_records<TA>(a, q, L, rhs);
    __syncthreads();
    const double lam = a.reg_mode ? a.lambda * (double)m : a.lambda;
    for (int k = tid; k < K; k += 256) L[k * (k + 1) / 2 + k] += lam;
    __syncthreads();

    // Cholesky L L^T of the packed lower triangle (text after Theorem 1),
    // right-looking in panels of 32 columns: the panel's diagonal block by
    // one wavefront, the rows below it one per thread, then the trailing
    // lower triangle in 4 x 4 tiles (three workgroup barriers per panel).
    __shared__ double rdiag[kFoldMaxKFull];
    __shared__ double col[kPanel];
    __shared__ int failed;
    const int wave = tid >> 6, lane = tid & 63;
    if (tid == 0) failed = 0;
    __syncthreads();
    for (int c0 = 0; c0 < K; c0 += kPanel) {
        const int w = K - c0 < kPanel ? K - c0 : kPanel;
        if (wave == 0) fold_diag_block(L, c0, w, rdiag, col, &failed);
        __syncthreads();
        fold_panel_rows(L, c0, w, K, rdiag);
        __syncthreads();
        fold_trailing(L, c0, w, K);
        __syncthreads();
    }
    if (tid == 0 && a.req_status) a.req_status[q] = failed ? TF_E_NUMERIC : TF_OK;
    if (failed) {
        if (tid == 0) atomicMin(a.bad_req, (unsigned long long)q);
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    // L y = c, then L^T a = y, by one wavefront with the unknowns in
    // registers (lane l holds unknowns l and l + 64): each solved value
    // reaches the lanes by a lane read, and every lane subtracts its
    // share; no barriers.
    if (wave != 0) return;
    const int l0 = lane, l1 = lane + 64;
    double y0 = l0 < K ? rhs[l0] : 0.0, y1 = l1 < K ? rhs[l1] : 0.0;
    for (int k = 0; k < K; ++k) {
        const double yk = (k < 64 ? lane_bcast(y0, k) : lane_bcast(y1, k - 64)) * rdiag[k];
        if (l0 == k) y0 = yk;
        if (l1 == k) y1 = yk;
        if (l0 > k && l0 < K) y0 -= L[tri(l0, k)] * yk;
        if (l1 > k && l1 < K) y1 -= L[tri(l1, k)] * yk;
    }
    for (int k = K - 1; k >= 0; --k) {
        const double ak = (k < 64 ? lane_bcast(y0, k) : lane_bcast(y1, k - 64)) * rdiag[k];
        if (l0 == k) y0 = ak;
        if (l1 == k) y1 = ak;
        if (l0 < k) y0 -= L[tri(k, l0)] * ak;
        if (l1 < k) y1 -= L[tri(k, l1)] * ak;
    }
    if (l0 < K) out[l0] = y0;
    if (l1 < K) out[l1] = y1;
}

// CDTF fold-in of one request per workgroup: a = 0, then `sweeps` passes
// over k = 0..K-1 of the C = 1 update a_k = sum_j rhat_j p_jk /
// (lambda_i + sum_j p_jk^2), rhat = r + a_k p_k, r = x - P a (Section 3.1).
// With B = P^T P and c = P^T x the numerator is c_k - sum_{k' != k} B_kk'
// a_k', so each update needs one dot product of length K against the
// request's B (in LDS) instead of two passes over its entries.  One
// wavefront does the sweeps (lane l holds a_l and a_{l+64}); the other
// wavefronts only help sum the chunk records.
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_cdtf(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    extern __shared__ double smem[];
    const int K = a.K;
    const int q = blockIdx.x;
    const int64_t m = a.req_ptr[q + 1] - a.req_ptr[q];
    double *out = a.rows + (int64_t)q * K;
    const int tid = threadIdx.x;
    if (tid == 0 && a.req_status) a.req_status[q] = TF_OK;   // no pivots in the C = 1 update
    if (m == 0) {
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    double *B = smem;                       // packed lower triangle
    double *c = B + K * (K + 1) / 2;        // K
    sum_chunk_records<TA>(a, q, B, c);
    __syncthreads();
    if (tid >= 64) return;
    const double lam = a.reg_mode ? a.lambda * (double)m : a.lambda;
    const int l0 = tid, l1 = tid + 64;
    double a0 = 0.0, a1 = 0.0;
    auto bidx = [](int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; };
    for (int s = 0; s < a.sweeps; ++s) {
        for (int k = 0; k < K; ++k) {
            // sum over k' != k of B_kk' a_k' (fixed order over the wavefront)
            double t = 0.0;
            if (l0 < K && l0 != k) t += B[bidx(k, l0)] * a0;
            if (l1 < K && l1 != k) t += B[bidx(k, l1)] * a1;
            t = wave_sum(t);
            const double bkk = B[k * (k + 1) / 2 + k];
            const double ak = (c[k] - t) / (lam + bkk);
            if (l0 == k) a0 = ak;
            if (l1 == k) a1 = ak;
        }
    }
    if (l0 < K) out[l0] = a0;
    if (l1 < K) out[l1] = a1;
}

// CDTF fold-in for K above the Gram path's limit: one workgroup per request
// walks the request's entries for every column (rhat = r + a_k p_k, the two
// sums, r = rhat - a_k p_k), with r in global memory.
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_cdtf_entries(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    __shared__ double scratch[8];
    extern __shared__ double smem[];
    const int K = a.K;
    const int q = blockIdx.x;
    const int64_t beg = a.req_ptr[q], end = a.req_ptr[q + 1];
    const int64_t m = end - beg;
    double *out = a.rows + (int64_t)q * K;
    const int tid = threadIdx.x;
    double *av = smem;           // K
    if (tid == 0 && a.req_status) a.req_status[q] = TF_OK;   // no pivots in the C = 1 update
    if (m == 0) {
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    for (int k = tid; k < K; k += 256) av[k] = 0.0;
    const TA *P = reinterpret_cast<const TA *>(a.P) + beg * K;
    double *r = a.r + beg;
    for (int64_t j = tid; j < m; j += 256) r[j] = a.vals[beg + j];
    const double lam = a.reg_mode ? a.lambda * (double)m : a.lambda;
    __syncthreads();
    for (int s = 0; s < a.sweeps; ++s) {
        for (int k = 0; k < K; ++k) {
            const double ak_old = av[k];
            double num = 0.0, den = 0.0;
            for (int64_t j = tid; j < m; j += 256) {
                const double p = (double)P[j * K + k];
                const double rh = r[j] + ak_old * p;
                num += rh * p;
                den += p * p;
            }
            fold_block_sum2(num, den, scratch);
            const double ak = num / (lam + den);
            // each thread updates the entries it summed, so r needs no barrier
            for (int64_t j = tid; j < m; j += 256) {
                const double p = (double)P[j * K + k];
                r[j] = (r[j] + ak_old * p) - ak * p;
            }
            if (tid == 0) av[k] = ak;
        }
        __syncthreads();
    }
    for (int k = tid; k < K; k += 256) out[k] = av[k];
}

size_t fold_full_lds(int K, int prec)
{
    (void)prec;
    return (size_t)(K * (K + 1) / 2 + K) * 8;
}

hipError_t launch_fold_validate(const FoldArgs &a, int64_t total, const int64_t *dims,
                                hipStream_t st)
{
    Dims8x d{};
    for (int n = 0; n < a.N; ++n) d.d[n] = dims[n];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_validate, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, total, d);
    return hipGetLastError();
}

hipError_t launch_fold_compute(int prec, const FoldArgs &a, int64_t total, int method,
                               hipStream_t st)
{
    if (total > 0) {
        const int64_t g = (total * a.K + 255) / 256;
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_p<P_F64>, dim3((unsigned)g), dim3(256), 0, st, a, total);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_p<P_F32>, dim3((unsigned)g), dim3(256), 0, st, a, total);
        else hipLaunchKernelGGL(k_fold_p<P_BF16>, dim3((unsigned)g), dim3(256), 0, st, a, total);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.nreq == 0) return hipSuccess;
    if (!fold_uses_gram(a.K)) {
        const size_t lds = (size_t)a.K * 8;
        if (lds > 65536) {
            const void *fn = prec == P_F64 ? (const void *)k_fold_cdtf_entries<P_F64>
                           : prec == P_F32 ? (const void *)k_fold_cdtf_entries<P_F32>
                                           : (const void *)k_fold_cdtf_entries<P_BF16>;
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_cdtf_entries<P_F64>, dim3(a.nreq), dim3(256), lds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_cdtf_entries<P_F32>, dim3(a.nreq), dim3(256), lds, st, a);
        else hipLaunchKernelGGL(k_fold_cdtf_entries<P_BF16>, dim3(a.nreq), dim3(256), lds, st, a);
        return hipGetLastError();
    }
    if (a.nchunks > 0) {
        const size_t glds = (size_t)FOLD_CHUNK * a.K * (prec == P_F64 ? 8 : 4);
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_gram<P_F64>, dim3(a.nchunks), dim3(256), glds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_gram<P_F32>, dim3(a.nchunks), dim3(256), glds, st, a);
        else hipLaunchKernelGGL(k_fold_gram<P_BF16>, dim3(a.nchunks), dim3(256), glds, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t lds = fold_full_lds(a.K, prec);
    const void *fn = method == 0
        ? (prec == P_F64 ? (const void *)k_fold_full<P_F64>
           : prec == P_F32 ? (const void *)k_fold_full<P_F32> : (const void *)k_fold_full<P_BF16>)
        : (prec == P_F64 ? (const void *)k_fold_cdtf<P_F64>
           : prec == P_F32 ? (const void *)k_fold_cdtf<P_F32> : (const void *)k_fold_cdtf<P_BF16>);
    if (lds > 65536) {
        // more than 64 KB of dynamic LDS must be allowed per kernel; the
        // attempt's error state is cleared so that it cannot be mistaken for
        // a launch failure below
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (method == 0) {
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_full<P_F64>, dim3(a.nreq), dim3(256), lds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_full<P_F32>, dim3(a.nreq), dim3(256), lds, st, a);
        else hipLaunchKernelGGL(k_fold_full<P_BF16>, dim3(a.nreq), dim3(256), lds, st, a);
    } else {
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_cdtf<P_F64>, dim3(a.nreq), dim3(256), lds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_cdtf<P_F32>, dim3(a.nreq), dim3(256), lds, st, a);
        else hipLaunchKernelGGL(k_fold_cdtf<P_BF16>, dim3(a.nreq), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

}  // namespace tfk
