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
// triangle of B then c.  FP32: on the matrix cores (below).  FP64: thread
// (ty, tx) accumulates rows ty + 16u and columns tx + 16v of B for the
// blocks v <= u that reach below row K.  (The
// entries' p rows come from k_fold_p, which forms them across the whole GPU:
// forming them here, chunk by chunk, made this kernel twice as slow.)
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_gram(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    __shared__ double xs[kFoldChunkEntries];
    extern __shared__ __align__(16) double smem[];
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
    if constexpr (PREC != P_F64) {
        // FP32 accumulation: B on the matrix cores.  The lower triangle's
        // 32 x 32 tiles (I >= J) go to the wavefronts in turn; one
        // v_mfma_f32_32x32x2f32 adds two entries' outer products to a tile:
        // lane c + 32h supplies column 32I + c (A) and 32J + c (B) of entry h
        // of the pair, and accumulator register r of lane c + 32h holds tile
        // element (8 (r / 4) + 4 h + r % 4, c).  c stays on the vector unit.
        typedef float f32x16 __attribute__((ext_vector_type(16)));
        const int wave = tid >> 6, lane = tid & 63, col = lane & 31, h = lane >> 5;
        const int nbk = (K + 31) / 32, ntile = nbk * (nbk + 1) / 2;
        // tile slots past the last tile compute tile 0 and are not stored,
        // so the entry loop has no branches (a branch around an accumulator
        // makes the compiler move it between register files every step)
        int ti[3], tj[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int t = wave + 4 * s < ntile ? wave + 4 * s : 0;
            int I = 0;
            while ((I + 1) * (I + 2) / 2 <= t) ++I;
            ti[s] = I;
            tj[s] = t - I * (I + 1) / 2;
        }
        f32x16 mac[3];
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int r = 0; r < 16; ++r) mac[s][r] = 0.f;
        // the whole chunk is staged at once (its loads all in flight together)
        {
            const int64_t c0 = beg;
            const int cn = (int)(end - beg);
            const TA *src = P + c0 * K;
            if ((K & 3) == 0) {
                const float4 *s4 = reinterpret_cast<const float4 *>(src);
                float4 *d4 = reinterpret_cast<float4 *>(Pc);
                for (int e = tid; e < cn * K / 4; e += 256) d4[e] = s4[e];
            } else {
                for (int e = tid; e < cn * K; e += 256) Pc[e] = src[e];
            }
            for (int e = tid; e < cn; e += 256) xs[e] = a.vals[c0 + e];
            __syncthreads();
            for (int j0 = 0; j0 < cn; j0 += 2) {
                const int e = j0 + h;
                const bool ein = e < cn;
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const int ka = 32 * ti[s] + col, kb = 32 * tj[s] + col;
                    const bool va = ein && ka < K, vb = ein && kb < K;
                    const float x = Pc[va ? e * K + ka : 0], y = Pc[vb ? e * K + kb : 0];
                    mac[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(va ? x : 0.f, vb ? y : 0.f,
                                                                 mac[s], 0, 0, 0);
                }
            }
            if (tid < K)
                for (int j = 0; j < cn; ++j) racc += (TA)xs[j] * Pc[j * K + tid];
        }
        TA *out = reinterpret_cast<TA *>(a.gpart) + (int64_t)cidx * fold_gram_stride(K);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (wave + 4 * s >= ntile) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int gi = 32 * ti[s] + 8 * (r / 4) + 4 * h + r % 4, gj = 32 * tj[s] + col;
                if (gi < K && gj <= gi) out[gi * (gi + 1) / 2 + gj] = mac[s][r];
            }
        }
        if (tid < K) out[K * (K + 1) / 2 + tid] = racc;
        return;
    }
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

constexpr int kPanel = 16;   // columns per panel of the blocked Cholesky

// 1 / sqrt(d) for d > 0: the hardware estimate and two steps of Newton's
// iteration r <- r (3 - d r^2) / 2, each roughly doubling the correct bits.
__device__ __forceinline__ double fold_rsqrt(double d)
{
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}

// 1 / d for d > 0: the hardware estimate and two steps of Newton's
// iteration r <- r + r (1 - d r), each roughly doubling the correct bits.
__device__ __forceinline__ double fold_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Width of a panel: WC columns when WC > 0 (a full panel, whose loop bounds
// are then known when compiling), else the run-time w.
template <int WC>
__device__ __forceinline__ int panel_w(int w) { return WC > 0 ? WC : w; }

// Cholesky of the diagonal block (rows and columns c0 .. c0 + w - 1, w <=
// 16) of the packed triangle, in place, by one wavefront: lane i holds row i
// of the block in registers.  Step j updates every row by M(i, k) -=
// f_i M(k, j) with f_i = M(i, j) / d_j (= L(i, j) L(k, j)), d_j the pivot.
// The loop carries only unscaled values, each step's chain being short:
// right after column j + 1 is updated, lane j + 1's new pivot reaches every
// lane by lane reads and each lane forms its next f beside the rest of the
// step's row updates, and lane k publishes M(k, j + 1) in colu[] for the next
// step's reads (two buffers; LDS accesses of one wavefront stay in program
// order).  Lane i's pivot stays in m[i]; afterwards it takes 1 / sqrt of it,
// publishes that as rdiag[c0 + i], and scales its row: L(i, j) = M(i, j) /
// sqrt(d_j), L(i, i) = sqrt(d_i).  A non-positive pivot sets *failed (the
// request is then reported and its row not used).  Lanes with no row, and
// registers k beyond a lane's row, are updated as scratch and never stored.
template <int WC>
__device__ __forceinline__ void fold_diag_block(double *L, int c0, int w_rt, double *rdiag,
                                                double (*colu)[64], int *failed)
{
    const int w = panel_w<WC>(w_rt);
    int i = threadIdx.x & 63;
    asm volatile("" : "+v"(i));   // lane tests stay in this call, not held across panels
    const bool in = i < w;
    double m[kPanel];
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const bool own = in && k <= i;
        const double v = L[own ? tri(c0 + i, c0 + k) : 0];
        m[k] = own ? v : 0.0;
    }
    colu[0][i] = m[0];
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    double cu[kPanel];
#pragma unroll
    for (int k = 1; k < kPanel; ++k) cu[k] = colu[0][k];
    double f = m[0] * fold_rcp(lane_bcast(m[0], 0));
#pragma unroll
    for (int j = 0; j < kPanel; ++j) {
        if (j >= w) continue;   // (not break: the loop must unroll fully)
        double fn = 0.0, cn[kPanel];
        if (j + 1 < w) {
            m[j + 1] -= f * cu[j + 1];
            colu[(j + 1) & 1][i] = m[j + 1];
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
#pragma unroll
            for (int k = j + 2; k < kPanel; ++k) cn[k] = colu[(j + 1) & 1][k];
            fn = m[j + 1] * fold_rcp(lane_bcast(m[j + 1], j + 1));
        }
#pragma unroll
        for (int k = j + 2; k < kPanel; ++k) m[k] -= f * cu[k];
#pragma unroll
        for (int k = j + 2; k < kPanel; ++k) cu[k] = cn[k];
        f = fn;
    }
    double di = 1.0;
#pragma unroll
    for (int k = 0; k < kPanel; ++k) di = k == i ? m[k] : di;
    const bool ok = !in || di > 0.0;
    const double rinv = fold_rsqrt(in ? di : 1.0);
    if (in) rdiag[c0 + i] = rinv;
    if (__ballot(!ok) != 0 && i == 0) *failed = 1;
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const double rk = rdiag[c0 + (k < w ? k : 0)];
        m[k] = k == i ? di * rinv : m[k] * rk;
    }
#pragma unroll
    for (int k = 0; k < kPanel; ++k)
        if (in && k <= i) L[tri(c0 + i, c0 + k)] = m[k];
}

// Rows below the diagonal block: L(r, c0..) = A(r, c0..) L11^{-T}, by
// forward substitution against the block, two lanes per row: lane h of the
// pair holds the row's columns 2u + h, sums its half of each dot product
// (two partial sums), and one lane swap adds the other half, so both lanes
// form the same x(k) (a + b and b + a are equal in floating point).
template <int WC>
__device__ __forceinline__ void fold_panel_rows(double *L, int c0, int w_rt, int K, const double *rdiag)
{
    constexpr int H = kPanel / 2;
    const int w = panel_w<WC>(w_rt);
    const int h = threadIdx.x & 1;
    for (int r = c0 + w + (int)(threadIdx.x >> 1); r < K; r += (int)(blockDim.x >> 1)) {
        const int base = tri(r, c0);
        double xs[H];
#pragma unroll
        for (int u = 0; u < H; ++u) {
            const bool in = 2 * u + h < w;
            const double v = L[base + (in ? 2 * u + h : 0)];
            xs[u] = in ? v : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kPanel; ++k) {
            if (k >= w) continue;
            const int bk = tri(c0 + k, c0);
            double p[2] = {0.0, 0.0};
#pragma unroll
            for (int u = 0; 2 * u + 1 < k + 1; ++u) {
                // column 2u + h < k: lane 1 of the pair has one term fewer when k is odd
                const bool in = 2 * u + h < k;
                const double l = L[bk + (in ? 2 * u + h : 0)];
                p[u & 1] -= xs[u] * (in ? l : 0.0);
            }
            double part = p[0] + p[1];
            part += dpp_mov<0xB1>(part);
            const double own = (k & 1) == h ? xs[k >> 1] : 0.0;
            const double a = own + dpp_mov<0xB1>(own);   // A(r, c0 + k), from the lane that holds it
            const double xk = (a + part) * rdiag[c0 + k];
            if ((k & 1) == h) xs[k >> 1] = xk;
        }
#pragma unroll
        for (int u = 0; u < H; ++u)
            if (2 * u + h < w) L[base + 2 * u + h] = xs[u];
    }
}

// Trailing update of the rows and columns after the panel, in 4 x 4 tiles
// of the lower triangle: A(r, s) -= sum_k L(r, k) L(s, k) over the panel.
// A tile's rows past K read row K - 1 instead (those sums are not stored),
// so the 32 reads of each group of four columns are issued together.
template <int WC>
__device__ __forceinline__ void fold_trailing(double *L, int c0, int w_rt, int K)
{
    const int w = panel_w<WC>(w_rt);
    const int c1 = c0 + w, n = K - c1;
    if (n <= 0) return;
    const int T = (n + 3) / 4, ntile = T * (T + 1) / 2;
    for (int t = threadIdx.x; t < ntile; t += blockDim.x) {
        int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        const int tj = t - ti * (ti + 1) / 2;
        const int r0 = c1 + 4 * ti, s0 = c1 + 4 * tj;
        int br[4], bs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            br[u] = tri(r0 + u < K ? r0 + u : K - 1, c0);
            bs[u] = tri(s0 + u < K ? s0 + u : K - 1, c0);
        }
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 1
        for (int k0 = 0; k0 < w; k0 += 4) {
            double ra[4][4], sb[4][4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const bool kin = WC > 0 || k0 + kk < w;
                const int k = kin ? k0 + kk : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double a = L[br[u] + k], b = L[bs[u] + k];
                    ra[kk][u] = kin ? a : 0.0;
                    sb[kk][u] = kin ? b : 0.0;
                }
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += ra[kk][u] * sb[kk][v];
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

// One panel of the blocked Cholesky: its diagonal block by wavefront 0, the
// rows below it by lane pairs, then the trailing lower triangle.
template <int WC>
__device__ __forceinline__ void fold_panel(double *L, int c0, int w, int K, double *rdiag,
                                           double (*colu)[64], int *failed)
{
    if ((threadIdx.x >> 6) == 0) fold_diag_block<WC>(L, c0, w, rdiag, colu, failed);
    __syncthreads();
    fold_panel_rows<WC>(L, c0, w, K, rdiag);
    __syncthreads();
    fold_trailing<WC>(L, c0, w, K);
    __syncthreads();
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
    // LDS: packed lower triangle L (K(K+1)/2 doubles), then rhs (K doubles
    // and one spare): rhs is row K of the triangle, so the factorisation
    // carries c along and leaves y = L^-1 c there
    double *L = smem;
    double *rhs = L + K * (K + 1) / 2;
    sum_chunk_records<TA>(a, q, L, rhs);
    __syncthreads();
    const double lam = a.reg_mode ? a.lambda * (double)m : a.lambda;
    for (int k = tid; k < K; k += 256) L[k * (k + 1) / 2 + k] += lam;
    __syncthreads();

    // Cholesky L L^T of the packed lower triangle (text after Theorem 1),
    // right-looking in panels of 16 columns: the panel's diagonal block by
    // one wavefront, the rows below it by lane pairs, then the trailing
    // lower triangle in 4 x 4 tiles (three workgroup barriers per panel).
    __shared__ double rdiag[kFoldMaxKFull];
    __shared__ double colu[2][64];
    __shared__ int failed;
    const int wave = tid >> 6, lane = tid & 63;
    if (tid == 0) failed = 0;
    __syncthreads();
    for (int c0 = 0; c0 < K; c0 += kPanel) {
        const int w = K - c0 < kPanel ? K - c0 : kPanel;
        if (w == kPanel) fold_panel<kPanel>(L, c0, w, K + 1, rdiag, colu, &failed);
        else fold_panel<0>(L, c0, w, K + 1, rdiag, colu, &failed);
    }
    if (tid == 0 && a.req_status) a.req_status[q] = failed ? TF_E_NUMERIC : TF_OK;
    if (failed) {
        if (tid == 0) atomicMin(a.bad_req, (unsigned long long)q);
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    // L y = c came with the factorisation: c is row K of the packed
    // triangle (the rhs array), so the panel rows and trailing updates
    // turned it into y.  L^T a = y by one wavefront with the unknowns in
    // registers (lane l holds unknowns l and l + 64, and their pivots'
    // reciprocals): each solved value reaches the lanes by a lane read, and
    // every lane subtracts its share; no barriers.  The factor's entries
    // are read eight columns at a time ahead of the steps that use them.
    if (wave != 0) return;
    const int l0 = lane, l1 = lane + 64;
    const int K0 = K < 64 ? K : 64;
    const double rd0 = l0 < K ? rdiag[l0] : 0.0, rd1 = l1 < K ? rdiag[l1] : 0.0;
    double y0 = l0 < K ? rhs[l0] : 0.0, y1 = l1 < K ? rhs[l1] : 0.0;
    constexpr int SB = 8;
    // both loops unrolled over the largest K, so that every lane read names
    // its lane when compiling; columns from K up are skipped
#pragma unroll
    for (int kb = kFoldMaxKFull - 1; kb >= 64; kb -= SB) {
        if (kb - SB + 1 >= K) continue;
        double b0[SB], b1[SB];
#pragma unroll
        for (int t = 0; t < SB; ++t) {
            const int k = kb - t;
            const bool v0 = k >= 64 && k < K, v1 = v0 && l1 < k;
            const double e0 = L[v0 ? tri(k, l0) : 0], e1 = L[v1 ? tri(k, l1) : 0];
            b0[t] = v0 ? e0 : 0.0;
            b1[t] = v1 ? e1 : 0.0;
        }
#pragma unroll
        for (int t = 0; t < SB; ++t) {
            const int k = kb - t;
            if (k < 64 || k >= K) continue;
            const double ak = lane_bcast(y1 * rd1, k - 64);
            if (l1 == k) y1 = ak;
            y0 -= b0[t] * ak;
            y1 -= b1[t] * ak;
        }
    }
#pragma unroll
    for (int kb = 63; kb >= 0; kb -= SB) {
        if (kb - SB + 1 >= K0) continue;
        double b0[SB];
#pragma unroll
        for (int t = 0; t < SB; ++t) {
            const int k = kb - t;
            const bool v0 = k < K0 && l0 < k;
            const double e0 = L[v0 ? tri(k, l0) : 0];
            b0[t] = v0 ? e0 : 0.0;
        }
#pragma unroll
        for (int t = 0; t < SB; ++t) {
            const int k = kb - t;
            if (k >= K0) continue;
            const double ak = lane_bcast(y0 * rd0, k);
            if (l0 == k) y0 = ak;
            y0 -= b0[t] * ak;
        }
    }
    if (l0 < K) out[l0] = y0;
    if (l1 < K) out[l1] = y1;
}

// CDTF fold-in of one request per workgroup: a = 0, then `sweeps` passes
// over k = 0..K-1 of the C = 1 update a_k = sum_j rhat_j p_jk /
// (lambda_i + sum_j p_jk^2), rhat = r + a_k p_k, r = x - P a (Section 3.1).
// With B = P^T P and c = P^T x the numerator is c_k - sum_{k' != k} B_kk'
// a_k' = g_k + B_kk a_k, where g = c - B a (= P^T r) is kept up to date:
// when a_k changes by delta, every g_i loses delta B_ik.  So an update needs
// two lane reads (g_k, a_k) and one vector update instead of a sum over the
// request's entries or over the wavefront.  One wavefront does the sweeps
// (lane l holds a_l, g_l and a_{l+64}, g_{l+64}), reading the columns of B
// eight coordinates ahead; the other wavefronts only help sum the chunk
// records.
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_cdtf(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    extern __shared__ double smem[];
    __shared__ double bdiag[kFoldMaxKFull], rden[kFoldMaxKFull];
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
    for (int k = tid; k < K; k += 64) {
        const double bkk = B[tri(k, k)];
        bdiag[k] = bkk;
        rden[k] = 1.0 / (lam + bkk);
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    const int l0 = tid, l1 = tid + 64;
    double a0 = 0.0, a1 = 0.0;
    double g0 = l0 < K ? c[l0] : 0.0, g1 = l1 < K ? c[l1] : 0.0;
    auto bidx = [](int i, int j) { return i >= j ? tri(i, j) : tri(j, i); };
    constexpr int SB = 8;
    for (int s = 0; s < a.sweeps; ++s) {
        // unrolled over the largest K, so that every lane read names its lane
        // when compiling
#pragma unroll
        for (int kb = 0; kb < kFoldMaxKFull; kb += SB) {
            if (kb >= K) continue;
            double e0[SB], e1[SB], bk[SB], rk[SB];
#pragma unroll
            for (int t = 0; t < SB; ++t) {
                const int k = kb + t;
                const bool kin = k < K, v0 = kin && l0 < K, v1 = kin && l1 < K;
                const double x0 = B[v0 ? bidx(l0, k) : 0], x1 = B[v1 ? bidx(l1, k) : 0];
                e0[t] = v0 ? x0 : 0.0;
                e1[t] = v1 ? x1 : 0.0;
                bk[t] = bdiag[kin ? k : 0];
                rk[t] = rden[kin ? k : 0];
            }
#pragma unroll
            for (int t = 0; t < SB; ++t) {
                const int k = kb + t;
                if (k >= K) continue;
                const double gk = k < 64 ? lane_bcast(g0, k) : lane_bcast(g1, k - 64);
                const double ak0 = k < 64 ? lane_bcast(a0, k) : lane_bcast(a1, k - 64);
                const double ak = (gk + bk[t] * ak0) * rk[t];
                const double delta = ak - ak0;
                if (l0 == k) a0 = ak;
                if (l1 == k) a1 = ak;
                g0 -= delta * e0[t];
                g1 -= delta * e1[t];
            }
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
    return (size_t)(K * (K + 1) / 2 + K + 1) * 8;
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
        // FP64 stages FOLD_CHUNK entries at a time, FP32 a whole chunk (up to
        // 128 KB for K = 128, beyond the default 64 KB of dynamic LDS)
        const size_t glds = prec == P_F64 ? (size_t)FOLD_CHUNK * a.K * 8
                                          : (size_t)kFoldChunkEntries * a.K * 4;
        if (glds > 65536) {
            const void *fn = prec == P_F32 ? (const void *)k_fold_gram<P_F32>
                                           : (const void *)k_fold_gram<P_BF16>;
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
            (void)hipGetLastError();
            if (e != hipSuccess) return e;
        }
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
