// Residual evaluation on the mode copies, the loss of eq. (TF), and
// prediction (arXiv:1410.5209: eq. (TF), eq. (SALS_R)).
//
// The mode copies hold R-hat of the last split (x minus every column outside
// that split), so the true residual is r = rhat - sum_{c in last split}
// prod_n a^(n) (eq. (SALS_R)); every kernel here forms it on the fly.
// Reductions are deterministic: fixed work per block, fixed trees.
#include "dev_common.h"

namespace tfk {

// Row slot of this lane in a task (same mapping as the accumulation kernel).
struct Slot {
    int row;
    int64_t beg, end;
    int G, sub;
};

__device__ __forceinline__ Slot task_slot(const Task *tasks, const int32_t *items,
                                          const Chunk *chunks, const int32_t *rowptr, int t,
                                          int lane)
{
    const Task task = tasks[t];
    Slot s;
    s.G = task.G;
    const int lg = __ffs(task.G) - 1;
    const int grp = lane >> lg;
    s.sub = lane & (task.G - 1);
    s.row = -1;
    s.beg = s.end = 0;
    if (task.kind == 0) {
        if (grp < task.count) {
            s.row = items[task.base + grp];
            s.beg = rowptr[s.row];
            s.end = rowptr[s.row + 1];
        }
    } else {
        const Chunk c = chunks[task.base];
        s.row = c.row;
        s.beg = c.beg;
        s.end = c.end;
    }
    return s;
}

__device__ __forceinline__ double block_sum_256(double v)
{
    __shared__ double ws[4];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    __syncthreads();
    return s;
}

// Storage elements per 16-byte vector, and one vector of a row as FP64.
template <typename TS> struct EvalVec;
template <> struct EvalVec<double> {
    static constexpr int W = 2;
    __device__ static void load(const double *p, double (&o)[2])
    {
        const double2 t = *reinterpret_cast<const double2 *>(p);
        o[0] = t.x; o[1] = t.y;
    }
};
template <> struct EvalVec<float> {
    static constexpr int W = 4;
    __device__ static void load(const float *p, double (&o)[4])
    {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    }
};
template <> struct EvalVec<bf16> {
    static constexpr int W = 8;
    __device__ static void load(const bf16 *p, double (&o)[8])
    {
        const uint4 t = *reinterpret_cast<const uint4 *>(p);
        const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            o[2 * h] = (double)__uint_as_float(w[h] << 16);
            o[2 * h + 1] = (double)__uint_as_float(w[h] & 0xffff0000u);
        }
    }
};

// Sum of r^2 over the mode-0 copy (per block), optionally writing r in input
// order.  The pending columns of every gathered row are read with 16-byte
// vectors from the slab row start (the slab is laid out for their count, so
// whole vectors stay inside the row); products and sums in FP64.
template <int PREC>
__global__ __launch_bounds__(256) void k_eval_resid(EvalArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    using V = EvalVec<TS>;
    constexpr int MAXC = kMaxC;
    constexpr int NV = MAXC / V::W;
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    double se = 0.0;
    if (t < a.ntasks) {
        const Slot s = task_slot(a.tasks, a.items, a.chunks, a.rowptr, t, lane);
        const TR *rh = reinterpret_cast<const TR *>(a.rhat);
        const int np = a.npend;
        double own[MAXC];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double x[V::W];
            if (v * V::W < np && s.row >= 0)
                V::load(reinterpret_cast<const TS *>(a.Pown) + (int64_t)s.row * a.ld + v * V::W, x);
            else {
#pragma unroll
                for (int e = 0; e < V::W; ++e) x[e] = 0.0;
            }
#pragma unroll
            for (int e = 0; e < V::W; ++e) own[v * V::W + e] = x[e];
        }
        for (int64_t j = s.beg + s.sub; j < s.end; j += s.G) {
            double prod[MAXC];
#pragma unroll
            for (int c = 0; c < MAXC; ++c) prod[c] = own[c];
            for (int l = 0; l < a.no; ++l) {
                const TS *row = reinterpret_cast<const TS *>(a.P[l]) + (int64_t)a.oidx[l][j] * a.ld;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (v * V::W < np) {
                        double x[V::W];
                        V::load(row + v * V::W, x);
#pragma unroll
                        for (int e = 0; e < V::W; ++e) prod[v * V::W + e] *= x[e];
                    }
                }
            }
            double r = (double)rh[j];
#pragma unroll
            for (int c = 0; c < MAXC; ++c)
                if (c < np) r -= prod[c];
            se += r * r;
            if (a.r_out) a.r_out[a.perm[j]] = r;
        }
    }
    const double tot = block_sum_256(se);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = tot;
}

hipError_t launch_eval_residual(int prec, const EvalArgs &a, int grid, hipStream_t st)
{
    if (prec == P_F64) hipLaunchKernelGGL(k_eval_resid<P_F64>, dim3(grid), dim3(256), 0, st, a);
    else if (prec == P_F32) hipLaunchKernelGGL(k_eval_resid<P_F32>, dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_eval_resid<P_BF16>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Per-block sums of w_i * ||a_i||^2 (w_i = 1, or the row count when weighted).
template <int PREC>
__global__ __launch_bounds__(256) void k_reg(const void *A, int64_t I, int K, const int32_t *rowptr,
                                             int weighted, double *partials)
{
    using TS = typename Types<PREC>::TS;
    const int64_t per = (I + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < I ? r0 + per : I;
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) {
            const double v = load_f64(reinterpret_cast<const TS *>(A) + i * K + k);
            s += v * v;
        }
        const double w = weighted ? (double)(rowptr[i + 1] - rowptr[i]) : 1.0;
        acc += w * s;
    }
    const double tot = block_sum_256(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

hipError_t reg_partials(int prec, const void *A, int64_t I, int K, const int32_t *rowptr,
                        int weighted, double *partials, int nblocks, hipStream_t st)
{
    if (prec == P_F64) hipLaunchKernelGGL(k_reg<P_F64>, dim3(nblocks), dim3(256), 0, st, A, I, K, rowptr, weighted, partials);
    else if (prec == P_F32) hipLaunchKernelGGL(k_reg<P_F32>, dim3(nblocks), dim3(256), 0, st, A, I, K, rowptr, weighted, partials);
    else hipLaunchKernelGGL(k_reg<P_BF16>, dim3(nblocks), dim3(256), 0, st, A, I, K, rowptr, weighted, partials);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sum(const double *p, int64_t n, double *out)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
    const double tot = block_sum_256(s);
    if (threadIdx.x == 0) *out = tot;
}

hipError_t sum_partials(const double *partials, int64_t n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, partials, n, out);
    return hipGetLastError();
}

struct PredPtrs { const void *A[kMaxModes]; int64_t dims[kMaxModes]; };

// x-hat = sum_k prod_n a^(n)_{i_n k}; one thread per query.
template <int PREC>
__global__ void k_predict(int N, int K, PredPtrs F, const int32_t *q, int64_t m, double *out,
                          unsigned long long *bad)
{
    using TS = typename Types<PREC>::TS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    int32_t ix[kMaxModes];
    bool okq = true;
    for (int n = 0; n < N; ++n) {
        ix[n] = q[t * N + n];
        okq = okq && ix[n] >= 0 && (int64_t)ix[n] < F.dims[n];
    }
    if (!okq) {
        atomicMin(bad, (unsigned long long)t);
        return;
    }
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
        double prod = 1.0;
        for (int n = 0; n < N; ++n)
            prod *= load_f64(reinterpret_cast<const TS *>(F.A[n]) + (int64_t)ix[n] * K + k);
        s += prod;
    }
    out[t] = s;
}

hipError_t launch_predict(int prec, int N, int K, const void *const *A, const int64_t *dims,
                          const int32_t *q, int64_t m, double *out, unsigned long long *bad,
                          hipStream_t st)
{
    PredPtrs F{};
    for (int n = 0; n < N; ++n) { F.A[n] = A[n]; F.dims[n] = dims[n]; }
    const int64_t grid = (m + 255) / 256;
    if (prec == P_F64) hipLaunchKernelGGL(k_predict<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, N, K, F, q, m, out, bad);
    else if (prec == P_F32) hipLaunchKernelGGL(k_predict<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, N, K, F, q, m, out, bad);
    else hipLaunchKernelGGL(k_predict<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, N, K, F, q, m, out, bad);
    return hipGetLastError();
}

// After a pass's solves: raise the sweep's stop flag if any mode recorded a
// non-positive pivot (see pass_halted).
__global__ void k_pass_latch(unsigned long long *flags, int nmodes)
{
    if (threadIdx.x != 0) return;
    bool any = false;
    for (int n = 0; n < nmodes; ++n) any = any || flags[n] != ~0ull;
    if (any) flags[kStopWord] = 1ull;
}

// Zero one counter word (a kernel, so that captured sweeps hold no memset).
__global__ void k_clear_word(unsigned int *p)
{
    if (threadIdx.x == 0) p[0] = 0u;
}

hipError_t launch_clear_word(unsigned int *p, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_pass_latch(unsigned long long *flags, int nmodes, hipStream_t st)
{
    hipLaunchKernelGGL(k_pass_latch, dim3(1), dim3(64), 0, st, flags, nmodes);
    return hipGetLastError();
}

}  // namespace tfk
