// Fold-in of new rows against resident factors (a use of the row update of
// arXiv:1410.5209 that the paper does not make itself): a request is a new
// row of one mode given by its observed entries (indices of the other modes
// and values).  Full rank solves eq. (ALS) for the row, a = (B + lambda_i I)^-1 c
// with c built from the values; CDTF runs coordinate sweeps of the C = 1
// update starting from a = 0.  One workgroup owns one request, so a request's
// result does not depend on the batch it travels in.
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

// Deterministic sum over a 256-thread block (fixed tree).
__device__ __forceinline__ double fold_block_sum(double v, double *scratch)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    return (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
}

constexpr int FOLD_CHUNK = 32;   // entries staged per step
constexpr int FOLD_RB = 8;       // register block per thread (8 x 8 -> K <= 128)

// Full-rank fold-in of one request per workgroup (K <= 128).
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
        return;
    }
    // LDS: packed lower triangle L (K(K+1)/2 doubles), rhs (K doubles),
    // staged P chunk (FOLD_CHUNK x K of TA), staged values, reduction scratch.
    double *L = smem;
    double *rhs = L + K * (K + 1) / 2;
    double *xs = rhs + K;
    double *scratch = xs + FOLD_CHUNK;
    TA *Pc = reinterpret_cast<TA *>(scratch + 8);

    const int ty = tid >> 4, tx = tid & 15;
    TA acc[FOLD_RB][FOLD_RB];
#pragma unroll
    for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
        for (int v = 0; v < FOLD_RB; ++v) acc[u][v] = TA(0);
    double racc = 0.0;   // rhs entry k = tid (tid < K)

    const TA *P = reinterpret_cast<const TA *>(a.P);
    for (int64_t c0 = beg; c0 < end; c0 += FOLD_CHUNK) {
        const int cn = (int)(end - c0 < FOLD_CHUNK ? end - c0 : FOLD_CHUNK);
        for (int e = tid; e < cn * K; e += 256) Pc[e] = P[c0 * K + e];
        if (tid < cn) xs[tid] = a.vals[c0 + tid];
        __syncthreads();
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
            if (tid < K) racc += xs[j] * (double)Pc[j * K + tid];
        }
        __syncthreads();
    }
    const double lam = a.reg_mode ? a.lambda * (double)m : a.lambda;
#pragma unroll
    for (int u = 0; u < FOLD_RB; ++u)
#pragma unroll
        for (int v = 0; v < FOLD_RB; ++v) {
            const int k1 = ty + 16 * u, k2 = tx + 16 * v;
            if (k1 < K && k2 <= k1) L[k1 * (k1 + 1) / 2 + k2] = (double)acc[u][v] + (k1 == k2 ? lam : 0.0);
        }
    if (tid < K) rhs[tid] = racc;
    __syncthreads();

    // Cholesky L L^T of the packed lower triangle (text after Theorem 1)
    __shared__ int failed;
    if (tid == 0) failed = 0;
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        if (tid == 0) {
            const double d = L[j * (j + 1) / 2 + j];
            if (!(d > 0.0)) failed = 1;
            L[j * (j + 1) / 2 + j] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        const double ljj = L[j * (j + 1) / 2 + j];
        for (int i = j + 1 + tid; i < K; i += 256) L[i * (i + 1) / 2 + j] /= ljj;
        __syncthreads();
        // trailing update of rows/columns j+1..K-1 (lower triangle, flattened)
        const int n = K - j - 1;
        const int T = n * (n + 1) / 2;
        for (int p = tid; p < T; p += 256) {
            int r = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= p) ++r;
            while (r * (r + 1) / 2 > p) --r;
            const int cidx = p - r * (r + 1) / 2;
            const int i = j + 1 + r, k = j + 1 + cidx;
            L[i * (i + 1) / 2 + k] -= L[i * (i + 1) / 2 + j] * L[k * (k + 1) / 2 + j];
        }
        __syncthreads();
    }
    if (failed) {
        if (tid == 0) atomicMin(a.bad_req, (unsigned long long)q);
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
    // L y = rhs (column sweep), then L^T a = y
    for (int k = 0; k < K; ++k) {
        if (tid == 0) rhs[k] = rhs[k] / L[k * (k + 1) / 2 + k];
        __syncthreads();
        const double yk = rhs[k];
        for (int i = k + 1 + tid; i < K; i += 256) rhs[i] -= L[i * (i + 1) / 2 + k] * yk;
        __syncthreads();
    }
    for (int k = K - 1; k >= 0; --k) {
        if (tid == 0) rhs[k] = rhs[k] / L[k * (k + 1) / 2 + k];
        __syncthreads();
        const double ak = rhs[k];
        for (int i = tid; i < k; i += 256) rhs[i] -= L[k * (k + 1) / 2 + i] * ak;
        __syncthreads();
    }
    for (int k = tid; k < K; k += 256) out[k] = rhs[k];
}

// CDTF fold-in of one request per workgroup: a = 0, r = x, then `sweeps`
// passes over k = 0..K-1 of rhat = r + a_k p_k; a_k = sum rhat p_k /
// (lambda_i + sum p_k^2); r = rhat - a_k p_k.
template <int PREC>
__global__ __launch_bounds__(256) void k_fold_cdtf(FoldArgs a)
{
    using TA = typename Types<PREC>::TA;
    extern __shared__ double smem[];
    const int K = a.K;
    const int q = blockIdx.x;
    const int64_t beg = a.req_ptr[q], end = a.req_ptr[q + 1];
    const int64_t m = end - beg;
    double *out = a.rows + (int64_t)q * K;
    const int tid = threadIdx.x;
    double *av = smem;           // K
    double *scratch = av + K;    // 8
    for (int k = tid; k < K; k += 256) av[k] = 0.0;
    if (m == 0) {
        for (int k = tid; k < K; k += 256) out[k] = 0.0;
        return;
    }
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
            num = fold_block_sum(num, scratch);
            den = fold_block_sum(den, scratch + 4);
            const double ak = num / (lam + den);
            for (int64_t j = tid; j < m; j += 256) {
                const double p = (double)P[j * K + k];
                r[j] = (r[j] + ak_old * p) - ak * p;
            }
            __syncthreads();
            if (tid == 0) av[k] = ak;
            __syncthreads();
        }
    }
    for (int k = tid; k < K; k += 256) out[k] = av[k];
}

size_t fold_full_lds(int K, int prec)
{
    const size_t ta = prec == P_F64 ? 8 : 4;
    return (size_t)(K * (K + 1) / 2 + K + FOLD_CHUNK + 8) * 8 + (size_t)FOLD_CHUNK * K * ta;
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
    if (method == 0) {
        const size_t lds = fold_full_lds(a.K, prec);
        if (lds > 65536) {
            // more than 64 KB of dynamic LDS must be allowed per kernel; the
            // attempt's error state is cleared so that it cannot be mistaken
            // for a launch failure below
            const void *fn = prec == P_F64 ? (const void *)k_fold_full<P_F64>
                           : prec == P_F32 ? (const void *)k_fold_full<P_F32>
                                           : (const void *)k_fold_full<P_BF16>;
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_full<P_F64>, dim3(a.nreq), dim3(256), lds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_full<P_F32>, dim3(a.nreq), dim3(256), lds, st, a);
        else hipLaunchKernelGGL(k_fold_full<P_BF16>, dim3(a.nreq), dim3(256), lds, st, a);
    } else {
        const size_t lds = (size_t)(a.K + 8) * 8;
        if (prec == P_F64) hipLaunchKernelGGL(k_fold_cdtf<P_F64>, dim3(a.nreq), dim3(256), lds, st, a);
        else if (prec == P_F32) hipLaunchKernelGGL(k_fold_cdtf<P_F32>, dim3(a.nreq), dim3(256), lds, st, a);
        else hipLaunchKernelGGL(k_fold_cdtf<P_BF16>, dim3(a.nreq), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

}  // namespace tfk
