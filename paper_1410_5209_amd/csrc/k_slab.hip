// Column slabs: the C columns of a split packed into an I x ld array per mode
// (only these columns are touched by a split -- memory theorem after the
// complexity analysis of arXiv:1410.5209), and written back at the end.
// Each slab row interleaves the current values W, the previous split's final
// values P and this split's start values S of one factor row.
#include "dev_common.h"

namespace tfk {

// Interleaved slab row of one factor row: [W | P | S], segments sw wide.
// W and S get the split's columns (zero past ncur), P the previous split's
// columns (zero past npend).  A block covers 256 / E rows, E (a power of two
// >= 3 sw, at most 256) threads per row, so a thread finds its row and
// element with shifts instead of 64-bit divisions.
template <typename TS>
__global__ __launch_bounds__(256) void k_pack(const TS *A, int64_t I, int K, const int32_t *cur,
                                              int ncur, const int32_t *pend, int npend, int sw,
                                              int64_t ld, int lgE, TS *Z)
{
    const int e = threadIdx.x & ((1 << lgE) - 1);
    const int64_t i = ((int64_t)blockIdx.x << (8 - lgE)) + (threadIdx.x >> lgE);
    if (i >= I || e >= 3 * sw) return;
    const int seg = e / sw;
    const int c = e - seg * sw;
    TS v = store_cast<TS>(0.0);
    if (seg == 1) {
        if (c < npend) v = A[i * K + pend[c]];
    } else if (c < ncur) {
        v = A[i * K + cur[c]];
    }
    Z[i * ld + e] = v;
}

// W of the split's columns back into the factor, E >= ncols threads per row.
template <typename TS>
__global__ __launch_bounds__(256) void k_unpack(const TS *W, int64_t I, int K, const int32_t *cols,
                                                int ncols, int64_t ld, int lgE, TS *A)
{
    const int c = threadIdx.x & ((1 << lgE) - 1);
    const int64_t i = ((int64_t)blockIdx.x << (8 - lgE)) + (threadIdx.x >> lgE);
    if (i >= I || c >= ncols) return;
    A[i * K + cols[c]] = W[i * ld + c];
}

namespace {
// log2 of the threads per row: the smallest power of two >= n (n <= 256)
int lg_threads(int n)
{
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    return lg;
}
}  // namespace

hipError_t pack_slab(int prec, const void *A, int64_t I, int K, const int32_t *cur, int ncur,
                     const int32_t *pend, int npend, int64_t sw, int64_t ld, void *Z, hipStream_t st)
{
    if (3 * sw > 256) return hipErrorInvalidValue;
    const int lgE = lg_threads((int)(3 * sw));
    const int64_t rows_per_block = (int64_t)1 << (8 - lgE);
    const int64_t grid = (I + rows_per_block - 1) / rows_per_block;
    const int s = (int)sw;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_pack<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)A, I, K, cur, ncur, pend, npend, s, ld, lgE, (double *)Z);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_pack<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)A, I, K, cur, ncur, pend, npend, s, ld, lgE, (float *)Z);
    else
        hipLaunchKernelGGL(k_pack<bf16>, dim3((unsigned)grid), dim3(256), 0, st, (const bf16 *)A, I, K, cur, ncur, pend, npend, s, ld, lgE, (bf16 *)Z);
    return hipGetLastError();
}

hipError_t unpack_slab(int prec, const void *W, int64_t I, int K, const int32_t *cols, int ncols,
                       int64_t ld, void *A, hipStream_t st)
{
    if (ncols > 256) return hipErrorInvalidValue;
    const int lgE = lg_threads(ncols);
    const int64_t rows_per_block = (int64_t)1 << (8 - lgE);
    const int64_t grid = (I + rows_per_block - 1) / rows_per_block;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_unpack<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)W, I, K, cols, ncols, ld, lgE, (double *)A);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_unpack<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)W, I, K, cols, ncols, ld, lgE, (float *)A);
    else
        hipLaunchKernelGGL(k_unpack<bf16>, dim3((unsigned)grid), dim3(256), 0, st, (const bf16 *)W, I, K, cols, ncols, ld, lgE, (bf16 *)A);
    return hipGetLastError();
}

}  // namespace tfk
