// Column slabs: the C columns of a split packed into an I x ld array per mode
// (only these columns are touched by a split -- memory theorem after the
// complexity analysis of arXiv:1410.5209), and written back at the end.
#include "dev_common.h"

namespace tfk {

template <typename TS>
__global__ void k_pack(const TS *A, int64_t I, int K, const int32_t *cols, int ncols, int CP,
                       int64_t ld, TS *o1, TS *o2)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= I * CP) return;
    const int64_t i = t / CP;
    const int c = (int)(t - i * CP);
    TS v;
    if (c < ncols) v = A[i * K + cols[c]];
    else v = store_cast<TS>(0.0);
    o1[i * ld + c] = v;
    if (o2) o2[i * ld + c] = v;
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

hipError_t pack_slab(int prec, const void *A, int64_t I, int K, const int32_t *cols, int ncols,
                     int CP, int64_t ld, void *out1, void *out2, hipStream_t st)
{
    const int64_t grid = (I * CP + 255) / 256;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_pack<double>, dim3((unsigned)grid), dim3(256), 0, st, (const double *)A, I, K, cols, ncols, CP, ld, (double *)out1, (double *)out2);
    else if (prec == P_F32)
        hipLaunchKernelGGL(k_pack<float>, dim3((unsigned)grid), dim3(256), 0, st, (const float *)A, I, K, cols, ncols, CP, ld, (float *)out1, (float *)out2);
    else
        hipLaunchKernelGGL(k_pack<bf16>, dim3((unsigned)grid), dim3(256), 0, st, (const bf16 *)A, I, K, cols, ncols, CP, ld, (bf16 *)out1, (bf16 *)out2);
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
