// One-time state construction: input validation, the mode-n CSR (a stable
// LSD radix sort of entry ids by row, 8-bit digits), the per-mode copies of
// the other-mode indices and of the residual, factor initialisation and the
// residual r = x - reconstruction (Section 3.1 of arXiv:1410.5209).
#include <climits>

#include "dev_common.h"

namespace tfk {

struct Dims8 { int64_t d[kMaxModes]; };

__global__ void k_validate(const int32_t *idx, const double *vals, int64_t nnz, int N, Dims8 dims,
                           unsigned long long *bad_idx, unsigned long long *bad_val)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    bool bad = false;
    for (int n = 0; n < N; ++n) {
        const int32_t v = idx[j * N + n];
        bad = bad || v < 0 || (int64_t)v >= dims.d[n];
    }
    if (bad) atomicMin(bad_idx, (unsigned long long)j);
    if (!isfinite(vals[j])) atomicMin(bad_val, (unsigned long long)j);
}

hipError_t validate_input(const int32_t *idx, const double *vals, int64_t nnz, int N,
                          const int64_t *dims, unsigned long long *bad_idx,
                          unsigned long long *bad_val, hipStream_t st)
{
    Dims8 d{};
    for (int n = 0; n < N; ++n) d.d[n] = dims[n];
    const int64_t grid = (nnz + 255) / 256;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)grid), dim3(256), 0, st, idx, vals, nnz, N, d,
                       bad_idx, bad_val);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

// Exclusive scan of one tile in place; the tile total goes to sums[block].
__global__ __launch_bounds__(SC_THREADS) void k_scan_tile(int32_t *data, int64_t n, int32_t *sums)
{
    __shared__ int32_t s[SC_THREADS];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int32_t v[SC_ITEMS];
    int32_t tot = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < n) ? data[base + i] : 0;
        const int32_t x = v[i];
        v[i] = tot;
        tot += x;
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < SC_THREADS; off <<= 1) {
        int32_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int32_t excl = s[threadIdx.x] - tot;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i)
        if (base + i < n) data[base + i] = v[i] + excl;
    if (threadIdx.x == SC_THREADS - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_add(int32_t *data, int64_t n, const int32_t *sums)
{
    const int32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    for (int i = threadIdx.x; i < SC_TILE; i += SC_THREADS)
        if (base + i < n) data[base + i] += add;
}

int64_t scan_tmp_size(int64_t n)
{
    int64_t tot = 0;
    while (n > 1) {
        n = (n + SC_TILE - 1) / SC_TILE;
        tot += n + 64;
    }
    return tot + 64;
}

static hipError_t exclusive_scan(int32_t *data, int64_t n, int32_t *tmp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SC_TILE - 1) / SC_TILE;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(SC_THREADS), 0, st, data, n, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = exclusive_scan(tmp, nb, tmp + nb + 64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SC_THREADS), 0, st, data, n, tmp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

int64_t sort_hist_size(int64_t nnz) { return 256 * ((nnz + RS_TILE - 1) / RS_TILE); }

// Digit histogram of one tile; hist is digit-major: hist[d * nblocks + b].
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const int32_t *keys, int64_t kstride,
                                                        int64_t n, int shift, int32_t *hist,
                                                        int nblocks)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = base + it * RS_THREADS + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e * kstride] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements keep their order among equal digits.  A tile is
// processed in rounds of 256 consecutive elements; inside a round an
// element's rank is (elements of earlier waves with its digit) + (lanes below
// it in its wave with its digit, found with ballots over the 8 digit bits).
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const int32_t *keys, int64_t kstride,
                                                           const int32_t *vals, int64_t n,
                                                           int shift, const int32_t *offs,
                                                           int nblocks, int32_t *okeys,
                                                           int32_t *ovals)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[RS_THREADS / 64][256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = base + it * RS_THREADS + tid;
        const bool valid = e < n;
        const int32_t key = valid ? keys[e * kstride] : 0;
        const int d = (key >> shift) & 255;
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = __popcll(same & below);
        const int cnt = __popcll(same);
        if (valid && rank == cnt - 1) wcnt[wave][d] = cnt;
        __syncthreads();
        int32_t pos = 0;
        if (valid) {
            pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < RS_THREADS / 64; ++w) { add += wcnt[w][tid]; wcnt[w][tid] = 0; }
        run[tid] += add;
        __syncthreads();
        if (valid) {
            okeys[pos] = key;
            ovals[pos] = vals ? vals[e] : (int32_t)e;
        }
    }
}

// Sorts entry ids by idx[j*N + mode] (keys < 2^key_bits), stably.
// Buffers: k0, k1, v1 (and perm_out as the other value buffer), nnz each.
// On return perm_out holds the sorted ids and k0 the sorted keys.
hipError_t stable_sort_by_key(const int32_t *idx, int N, int mode, int64_t nnz, int key_bits,
                              int32_t *perm_out, int32_t *k0, int32_t *k1, int32_t *v1,
                              int32_t *hist, int64_t hist_cap, int32_t *scan_tmp,
                              int64_t scan_tmp_cap, hipStream_t st)
{
    const int64_t nb = (nnz + RS_TILE - 1) / RS_TILE;
    if (256 * nb > hist_cap || scan_tmp_size(256 * nb) > scan_tmp_cap) return hipErrorInvalidValue;
    int passes = (key_bits + 7) / 8;
    if (passes < 1) passes = 1;
    // ping-pong so that the last pass writes keys to k0 and values to perm_out
    const int32_t *ksrc = idx + mode;
    int64_t kstride = N;
    const int32_t *vsrc = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool to_final = ((passes - 1 - p) % 2) == 0;
        int32_t *kdst = to_final ? k0 : k1;
        int32_t *vdst = to_final ? perm_out : v1;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, ksrc, kstride,
                           nnz, 8 * p, hist, (int)nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan(hist, 256 * nb, scan_tmp, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, ksrc,
                           kstride, vsrc, nnz, 8 * p, hist, (int)nb, kdst, vdst);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ksrc = kdst;
        kstride = 1;
        vsrc = vdst;
    }
    return hipSuccess;
}

__global__ void k_rowptr(const int32_t *sk, int64_t nnz, int64_t I, int32_t *rowptr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > nnz) return;
    const int64_t prev = (p > 0) ? (int64_t)sk[p - 1] : -1;
    const int64_t cur = (p < nnz) ? (int64_t)sk[p] : I;
    for (int64_t r = prev + 1; r <= cur && r <= I; ++r) rowptr[r] = (int32_t)p;
}

hipError_t rowptr_from_sorted(const int32_t *sorted_keys, int64_t nnz, int64_t I, int32_t *rowptr,
                              hipStream_t st)
{
    const int64_t grid = (nnz + 1 + 255) / 256;
    hipLaunchKernelGGL(k_rowptr, dim3((unsigned)grid), dim3(256), 0, st, sorted_keys, nnz, I, rowptr);
    return hipGetLastError();
}

__global__ void k_gather_idx(const int32_t *idx, int N, int l, const int32_t *perm, int64_t nnz,
                             int32_t *out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) out[p] = idx[(int64_t)perm[p] * N + l];
}

hipError_t gather_other_index(const int32_t *idx, int N, int l, const int32_t *perm, int64_t nnz,
                              int32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_idx, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, idx,
                       N, l, perm, nnz, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ factors
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) as a counter-based generator:
// output t for seed s is mix(s + t * 0x9E3779B97F4A7C15).  Entry (i, k) of
// factor n uses counter 1 + offset_n + i*K + k; value U(0,1) / sqrt(K).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int PREC>
__global__ void k_init_factor(void *A, int64_t I, int K, uint64_t seed, uint64_t offset, int zero)
{
    using TS = typename Types<PREC>::TS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= I * K) return;
    double v = 0.0;
    if (!zero) {
        const double u = (double)(splitmix64(seed, 1 + offset + (uint64_t)t) >> 11) *
                         (1.0 / 9007199254740992.0);
        v = u / sqrt((double)K);
    }
    reinterpret_cast<TS *>(A)[t] = store_cast<TS>(v);
}

hipError_t init_factor(int prec, void *A, int64_t I, int K, uint64_t seed, uint64_t offset,
                       bool zero, hipStream_t st)
{
    const int64_t grid = (I * K + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_init_factor<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, A, I, K, seed, offset, (int)zero);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_init_factor<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, A, I, K, seed, offset, (int)zero);
    else
        hipLaunchKernelGGL(k_init_factor<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, A, I, K, seed, offset, (int)zero);
    return hipGetLastError();
}

struct FactorPtrs { const void *A[kMaxModes]; };

// r_j = x_j - sum_k prod_n a^(n)_{i_n k}, in FP64, input order.
template <int PREC>
__global__ void k_residual(const int32_t *idx, const double *x, int64_t nnz, int N, FactorPtrs F,
                           int K, int zero_model, double *r)
{
    using TS = typename Types<PREC>::TS;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    double s = 0.0;
    if (!zero_model) {
        for (int k = 0; k < K; ++k) {
            double prod = 1.0;
            for (int n = 0; n < N; ++n)
                prod *= load_f64(reinterpret_cast<const TS *>(F.A[n]) + (int64_t)idx[j * N + n] * K + k);
            s += prod;
        }
    }
    r[j] = x[j] - s;
}

hipError_t residual_input_order(int prec, const int32_t *idx, const double *x, int64_t nnz, int N,
                                const void *const *A, int K, bool zero_model, double *r_out,
                                hipStream_t st)
{
    FactorPtrs F{};
    for (int n = 0; n < N; ++n) F.A[n] = A[n];
    const int64_t grid = (nnz + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_residual<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, idx, x, nnz, N, F, K, (int)zero_model, r_out);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_residual<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, idx, x, nnz, N, F, K, (int)zero_model, r_out);
    else
        hipLaunchKernelGGL(k_residual<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, idx, x, nnz, N, F, K, (int)zero_model, r_out);
    return hipGetLastError();
}

template <typename TR>
__global__ void k_gather_resid(const double *r, const int32_t *perm, int64_t nnz, TR *out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) out[p] = (TR)r[perm[p]];
}

hipError_t gather_residual(int prec, const double *r_in, const int32_t *perm, int64_t nnz,
                           void *rhat_out, hipStream_t st)
{
    const int64_t grid = (nnz + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_gather_resid<double>, dim3((unsigned)grid), dim3(256), 0, st, r_in, perm, nnz, (double *)rhat_out);
    else
        hipLaunchKernelGGL(k_gather_resid<float>, dim3((unsigned)grid), dim3(256), 0, st, r_in, perm, nnz, (float *)rhat_out);
    return hipGetLastError();
}

// Position in the mode-0 order of the entry at each position of another
// mode's order: inv[perm0[p]] = p, then out[q] = inv[permn[q]].
__global__ void k_invert_perm(const int32_t *perm, int64_t nnz, int32_t *inv)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) inv[perm[p]] = (int32_t)p;
}

__global__ void k_gather_i32(const int32_t *in, const int32_t *idx, int64_t nnz, int32_t *out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) out[q] = in[idx[q]];
}

hipError_t compose_with_mode0(const int32_t *perm0, const int32_t *permn, int64_t nnz,
                              int32_t *inv_scratch, int32_t *out, hipStream_t st)
{
    const int64_t grid = (nnz + 255) / 256;
    hipLaunchKernelGGL(k_invert_perm, dim3((unsigned)grid), dim3(256), 0, st, perm0, nnz, inv_scratch);
    hipLaunchKernelGGL(k_gather_i32, dim3((unsigned)grid), dim3(256), 0, st, inv_scratch, permn, nnz, out);
    return hipGetLastError();
}

template <typename TR>
__global__ void k_gather_copy(const TR *in, const int32_t *idx, int64_t nnz, TR *out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) out[q] = in[idx[q]];
}

hipError_t gather_copy(int prec, const void *in, const int32_t *idx, int64_t nnz, void *out,
                       hipStream_t st)
{
    const int64_t grid = (nnz + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_gather_copy<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)in, idx, nnz, (double *)out);
    else
        hipLaunchKernelGGL(k_gather_copy<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)in, idx, nnz, (float *)out);
    return hipGetLastError();
}

// A block of a factor as FP64: out[r * ncols + c] = A[row(r)][col(c)], where
// row(r) = rows[r] (r when rows is NULL) and col(c) = cols[c] (c when NULL).
template <int PREC>
__global__ void k_factor_block(const void *A, int K, const int32_t *rows, int64_t nrows,
                               const int32_t *cols, int ncols, double *out)
{
    using TS = typename Types<PREC>::TS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * ncols) return;
    const int64_t r = t / ncols;
    const int c = (int)(t - r * ncols);
    const int64_t i = rows ? rows[r] : r;
    const int k = cols ? cols[c] : c;
    out[t] = load_f64(reinterpret_cast<const TS *>(A) + i * K + k);
}

hipError_t factor_block_to_f64(int prec, const void *A, int K, const int32_t *rows,
                               int64_t nrows, const int32_t *cols, int ncols, double *out,
                               hipStream_t st)
{
    const int64_t grid = (nrows * ncols + 255) / 256;
    if (grid == 0) return hipSuccess;
    if (prec == P_F64) hipLaunchKernelGGL(k_factor_block<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, A, K, rows, nrows, cols, ncols, out);
    else if (prec == P_F32) hipLaunchKernelGGL(k_factor_block<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, A, K, rows, nrows, cols, ncols, out);
    else hipLaunchKernelGGL(k_factor_block<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, A, K, rows, nrows, cols, ncols, out);
    return hipGetLastError();
}

template <int PREC>
__global__ void k_to_f64(const void *A, int64_t n, double *out)
{
    using TS = typename Types<PREC>::TS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = load_f64(reinterpret_cast<const TS *>(A) + t);
}

template <int PREC>
__global__ void k_from_f64(const double *in, int64_t n, void *A)
{
    using TS = typename Types<PREC>::TS;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) reinterpret_cast<TS *>(A)[t] = store_cast<TS>(in[t]);
}

hipError_t factor_to_f64(int prec, const void *A, int64_t n, double *out, hipStream_t st)
{
    const int64_t grid = (n + 255) / 256;
    if (grid == 0) return hipSuccess;
    if (prec == P_F64) hipLaunchKernelGGL(k_to_f64<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, A, n, out);
    else if (prec == P_F32) hipLaunchKernelGGL(k_to_f64<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, A, n, out);
    else hipLaunchKernelGGL(k_to_f64<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, A, n, out);
    return hipGetLastError();
}

hipError_t factor_from_f64(int prec, const double *in, int64_t n, void *A, hipStream_t st)
{
    const int64_t grid = (n + 255) / 256;
    if (grid == 0) return hipSuccess;
    if (prec == P_F64) hipLaunchKernelGGL(k_from_f64<P_F64>, dim3((unsigned)grid), dim3(256), 0, st, in, n, A);
    else if (prec == P_F32) hipLaunchKernelGGL(k_from_f64<P_F32>, dim3((unsigned)grid), dim3(256), 0, st, in, n, A);
    else hipLaunchKernelGGL(k_from_f64<P_BF16>, dim3((unsigned)grid), dim3(256), 0, st, in, n, A);
    return hipGetLastError();
}

}  // namespace tfk
