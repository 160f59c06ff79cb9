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

// Partial Gram of one chunk of one request (full rank, K <= 128): B and c
// over the chunk's entries in the accumulation type, written as a record of
// the lower triangle of B then c.
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
            for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
                for (int v = 0; v < FOLD_RB; ++v) acc[u][v] += pr[u] * pc[v];
            if (tid < K) racc += (TA)xs[j] * Pc[j * K + tid];
        }
        __syncthreads();
    }
    TA *out = reinterpret_cast<TA *>(a.gpart) + (int64_t)cidx * fold_gram_stride(K);
#pragma unroll
    for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
        for (int v = 0; v < FOLD_RB; ++v) {
            const int k1 = ty + 16 * u, k2 = tx + 16 * v;
            if (k1 < K && k2 <= k1) out[k1 * (k1 + 1) / 2 + k2] = acc[u][v];
        }
    if (tid < K) out[K * (K + 1) / 2 + tid] = racc;
}

// B (packed lower triangle) and c of request q in FP64: its chunk records
// summed in chunk order (every thread of the block takes part).
template <typename TA>
__device__ __forceinline__ void sum_chunk_records(const FoldArgs &a, int q, double *L, double *rhs)
{
    const int K = a.K;
    const int KT = K * (K + 1) / 2;
    const int64_t gs = fold_gram_stride(K);
    const int c0 = a.chunk_first[q], nc = a.chunk_first[q + 1] - c0;
    const TA *gp = reinterpret_cast<const TA *>(a.gpart) + (int64_t)c0 * gs;
    for (int e = threadIdx.x; e < KT + K; e += blockDim.x) {
        double sum = 0.0;
        for (int t = 0; t < nc; ++t) sum += (double)gp[(int64_t)t * gs + e];
        if (e < KT) L[e] = sum;
        else rhs[e - KT] = sum;
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

    // Cholesky L L^T of the packed lower triangle (text after Theorem 1).
    // Each thread owns fixed positions p = tid + 256 t of the triangle, their
    // (row, column) decoded once; step j scales column j and updates the
    // owned elements right of it.  The diagonal of L goes to diag[].
    constexpr int kOwn = (kFoldMaxKFull * (kFoldMaxKFull + 1) / 2 + 255) / 256;
    __shared__ double diag[kFoldMaxKFull];
    __shared__ int failed;
    const int KT = K * (K + 1) / 2;
    int own[kOwn];
#pragma unroll
    for (int t = 0; t < kOwn; ++t) {
        const int p = tid + 256 * t;
        own[t] = -1;
        if (p < KT) {
            int r = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= p) ++r;
            while (r * (r + 1) / 2 > p) --r;
            own[t] = (r << 8) | (p - r * (r + 1) / 2);
        }
    }
    if (tid == 0) failed = 0;
    for (int j = 0; j < K; ++j) {
        __syncthreads();
        const double d = L[j * (j + 1) / 2 + j];
        const double ljj = sqrt(d > 0.0 ? d : 1.0), rinv = 1.0 / ljj;
        if (tid == 0) {
            diag[j] = ljj;
            if (!(d > 0.0)) failed = 1;
        }
        for (int i = j + 1 + tid; i < K; i += 256) L[i * (i + 1) / 2 + j] *= rinv;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kOwn; ++t) {
            const int i = own[t] >> 8, k = own[t] & 255;
            if (own[t] >= 0 && k > j)
                L[i * (i + 1) / 2 + k] -= L[i * (i + 1) / 2 + j] * L[k * (k + 1) / 2 + j];
        }
    }
    __syncthreads();
    if (tid == 0 && a.req_status) a.req_status[q] = failed ? TF_E_NUMERIC : TF_OK;
    if (failed) {
        if (tid == 0) atomicMin(a.bad_req, (unsigned long long)q);
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    // L y = rhs, then L^T a = y, by one wavefront (its LDS accesses stay in
    // program order, so no barriers)
    if (tid >= 64) return;
    for (int k = 0; k < K; ++k) {
        const double yk = rhs[k] / diag[k];
        __builtin_amdgcn_wave_barrier();
        for (int i = k + 1 + tid; i < K; i += 64) rhs[i] -= L[i * (i + 1) / 2 + k] * yk;
        if (tid == 0) rhs[k] = yk;
        __builtin_amdgcn_wave_barrier();
    }
    for (int k = K - 1; k >= 0; --k) {
        const double ak = rhs[k] / diag[k];
        __builtin_amdgcn_wave_barrier();
        for (int i = tid; i < k; i += 64) rhs[i] -= L[k * (k + 1) / 2 + i] * ak;
        if (tid == 0) rhs[k] = ak;
        __builtin_amdgcn_wave_barrier();
    }
    for (int k = tid; k < K; k += 64) out[k] = rhs[k];
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
            // sum over k' != k of B_kk' a_k' (fixed tree over the wavefront)
            double t = 0.0;
            if (l0 < K && l0 != k) t += B[bidx(k, l0)] * a0;
            if (l1 < K && l1 != k) t += B[bidx(k, l1)] * a1;
            for (int sh = 32; sh >= 1; sh >>= 1) t += __shfl_xor(t, sh, 64);
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
