// Device helpers shared by the kernels: storage types, row loads, rounding.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tf_internal.h"

namespace tfk {

// Storage / residual / accumulation types per precision.
template <int PREC> struct Types;
template <> struct Types<P_F64> { using TS = double; using TR = double; using TA = double; };
template <> struct Types<P_F32> { using TS = float;  using TR = float;  using TA = float; };
template <> struct Types<P_BF16> { using TS = bf16;  using TR = float;  using TA = float; };

// Elements per 16-byte vector of the storage type.
template <typename TS> struct VecW;
template <> struct VecW<double> { static constexpr int v = 2; };
template <> struct VecW<float> { static constexpr int v = 4; };
template <> struct VecW<bf16> { static constexpr int v = 8; };

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// float -> bf16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// double -> bf16, round to nearest even without double rounding: the double
// is first narrowed to float with round-to-odd (truncate toward zero, then
// set the last bit if anything was dropped), which keeps enough information
// for the final round-to-nearest-even step to 8 significant bits.
__device__ __forceinline__ uint16_t f64_to_bf16(double d)
{
    float f = (float)d;
    if (d != d) return f32_to_bf16(f);
    if (fabs((double)f) > fabs(d)) f = nextafterf(f, 0.0f);
    if ((double)f != d) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f32_to_bf16(f);
}

template <typename TS> __device__ __forceinline__ TS store_cast(double v);
template <> __device__ __forceinline__ double store_cast<double>(double v) { return v; }
template <> __device__ __forceinline__ float store_cast<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16 store_cast<bf16>(double v) { return bf16{f64_to_bf16(v)}; }

template <typename TS> __device__ __forceinline__ double load_f64(const TS *p);
template <> __device__ __forceinline__ double load_f64<double>(const double *p) { return *p; }
template <> __device__ __forceinline__ double load_f64<float>(const float *p) { return (double)*p; }
template <> __device__ __forceinline__ double load_f64<bf16>(const bf16 *p) { return (double)bf16_to_f32(p->bits); }

// Load CP consecutive storage elements (16-byte aligned row start; the slab
// stride is a multiple of the vector width, so whole vectors stay in bounds)
// and convert them to the accumulation type.
template <int CP, typename TA>
__device__ __forceinline__ void load_row(const double *__restrict__ p, TA (&out)[CP])
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int v = 0; v < (CP + 1) / 2; ++v) {
        double2 t = q[v];
        out[2 * v] = (TA)t.x;
        if (2 * v + 1 < CP) out[2 * v + 1] = (TA)t.y;
    }
}
template <int CP, typename TA>
__device__ __forceinline__ void load_row(const float *__restrict__ p, TA (&out)[CP])
{
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int v = 0; v < (CP + 3) / 4; ++v) {
        float4 t = q[v];
        out[4 * v] = (TA)t.x;
        if (4 * v + 1 < CP) out[4 * v + 1] = (TA)t.y;
        if (4 * v + 2 < CP) out[4 * v + 2] = (TA)t.z;
        if (4 * v + 3 < CP) out[4 * v + 3] = (TA)t.w;
    }
}
template <int CP, typename TA>
__device__ __forceinline__ void load_row(const bf16 *__restrict__ p, TA (&out)[CP])
{
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int v = 0; v < (CP + 7) / 8; ++v) {
        uint4 t = q[v];
        uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            if (8 * v + 2 * h < CP) out[8 * v + 2 * h] = (TA)__uint_as_float(w[h] << 16);
            if (8 * v + 2 * h + 1 < CP) out[8 * v + 2 * h + 1] = (TA)__uint_as_float(w[h] & 0xffff0000u);
        }
    }
}

template <typename T> __device__ __forceinline__ T stream_load(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void stream_store(T v, T *p) { __builtin_nontemporal_store(v, p); }

// Sum over the G lanes of a group (G a power of two, groups aligned).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G)
{
    for (int m = 1; m < G; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace tfk
