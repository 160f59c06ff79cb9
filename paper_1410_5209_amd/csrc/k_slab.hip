// Column slabs: the C columns of a split packed into an I x ld array per mode
// (only these columns are touched by a split -- memory theorem after the
// complexity analysis of arXiv:1410.5209), and written back at the end.
// Each slab row interleaves the current values W, the previous split's final
// values P and this split's start values S of one factor row.
#include "dev_common.h"

namespace tfk {

// Interleaved slab row of one factor row: [W | P | S], segments sw wide.
// W and S get the split's columns (zero past ncur), P the previous split's
// columns (zero past npend).
template <typename TS>
__global__ void k_pack(const TS *A, int64_t I, int K, const int32_t *cur, int ncur,
                       const int32_t *pend, int npend, int64_t sw, int64_t ld, TS *Z)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= I * 3 * sw) return;
    const int64_t i = t / (3 * sw);
    const int64_t e = t - i * 3 * sw;
    const int seg = (int)(e / sw);
    const int c = (int)(e - seg * sw);
    TS v = store_cast<TS>(0.0);
    if (seg == 1) {
        if (c < npend) v = A[i * K + pend[c]];
    } else if (c < ncur) {
        v = A[i * K + cur[c]];
    }
    Z[i * ld + e] = v;
}

template <typename TS>
__global__ void k_unpack(const TS *W, int64_t I, int K, const int32_t *cols, int ncols, int64_t ld,
                         TS *A)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= I * ncols) return;
    const int64_t i = t / ncols;
    const int c = (int)(t - i * ncols);
    A[i * K + cols[c]] = W[i * ld + c];
}

hipError_t pack_slab(int prec, const void *A, int64_t I, int K, const int32_t *cur, int ncur,
                     const int32_t *pend, int npend, int64_t sw, int64_t ld, void *Z, hipStream_t st)
{
    const int64_t grid = (I * 3 * sw + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_pack<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)A, I, K, cur, ncur, pend, npend, sw, ld, (double *)Z);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_pack<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)A, I, K, cur, ncur, pend, npend, sw, ld, (float *)Z);
    else
        hipLaunchKernelGGL(k_pack<bf16>, dim3((unsigned)grid), dim3(256), 0, st, (const bf16 *)A, I, K, cur, ncur, pend, npend, sw, ld, (bf16 *)Z);
    return hipGetLastError();
}

hipError_t unpack_slab(int prec, const void *W, int64_t I, int K, const int32_t *cols, int ncols,
                       int64_t ld, void *A, hipStream_t st)
{
    const int64_t grid = (I * ncols + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_unpack<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)W, I, K, cols, ncols, ld, (double *)A);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_unpack<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)W, I, K, cols, ncols, ld, (float *)A);
    else
        hipLaunchKernelGGL(k_unpack<bf16>, dim3((unsigned)grid), dim3(256), 0, st, (const bf16 *)W, I, K, cols, ncols, ld, (bf16 *)A);
    return hipGetLastError();
}

}  // namespace tfk
