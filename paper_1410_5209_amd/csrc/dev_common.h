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

// Same as load_row for a row start that is only 8-byte aligned (the
// pending-column segment of an interleaved slab row).
template <int CP, typename TA>
__device__ __forceinline__ void load_row8(const double *__restrict__ p, TA (&out)[CP])
{
#pragma unroll
    for (int c = 0; c < CP; ++c) out[c] = (TA)p[c];
}
template <int CP, typename TA>
__device__ __forceinline__ void load_row8(const float *__restrict__ p, TA (&out)[CP])
{
    const float2 *q = reinterpret_cast<const float2 *>(p);
#pragma unroll
    for (int v = 0; v < (CP + 1) / 2; ++v) {
        float2 t = q[v];
        out[2 * v] = (TA)t.x;
        if (2 * v + 1 < CP) out[2 * v + 1] = (TA)t.y;
    }
}
template <int CP, typename TA>
__device__ __forceinline__ void load_row8(const bf16 *__restrict__ p, TA (&out)[CP])
{
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
#pragma unroll
    for (int v = 0; v < (CP + 3) / 4; ++v) {
        uint2 t = q[v];
        uint32_t w[2] = {t.x, t.y};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (4 * v + 2 * h < CP) out[4 * v + 2 * h] = (TA)__uint_as_float(w[h] << 16);
            if (4 * v + 2 * h + 1 < CP) out[4 * v + 2 * h + 1] = (TA)__uint_as_float(w[h] & 0xffff0000u);
        }
    }
}

template <typename T> __device__ __forceinline__ T stream_load(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void stream_store(T v, T *p) { __builtin_nontemporal_store(v, p); }

// Cross-lane moves inside a row of 16 lanes (DPP, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// In-place sum over the G lanes of each aligned group (G a power of two, all
// 64 lanes active).  Inside 16 lanes: quad swaps (xor 1, xor 2), then the
// half-row and row mirrors, each pairing lanes from the two halves of the
// block summed so far; across rows: lane shuffles.  Every lane ends with its
// group's sum.
template <int NE, typename T>
__device__ __forceinline__ void group_reduce(T (&v)[NE], int G)
{
    if (G >= 2) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += dpp_mov<0xB1>(v[e]);   // quad_perm 1,0,3,2
    }
    if (G >= 4) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += dpp_mov<0x4E>(v[e]);   // quad_perm 2,3,0,1
    }
    if (G >= 8) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += dpp_mov<0x141>(v[e]);  // row_half_mirror
    }
    if (G >= 16) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += dpp_mov<0x140>(v[e]);  // row_mirror
    }
    if (G >= 32) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += __shfl_xor(v[e], 16, 64);
    }
    if (G >= 64) {
#pragma unroll
        for (int e = 0; e < NE; ++e) v[e] += __shfl_xor(v[e], 32, 64);
    }
}

// Persistent launches: the next task index for the calling wavefront (all
// 64 lanes active), taken by lane 0 from the launch's work counter.
__device__ __forceinline__ int take_task(unsigned int *work)
{
    int t = 0;
    if ((threadIdx.x & 63) == 0) t = (int)atomicAdd(work, 1u);
    return __shfl(t, 0, 64);
}

// A sweep stops updating factors after the first mode pass that meets a
// non-positive pivot (the rows of that pass that solved are kept), as the
// oracle's split loop does.  flags[0..kMaxModes) hold the smallest failing
// row per mode and flags[kStopWord] the sticky stop flag.  A solve launch
// reads the stop flag before any write (pass_halted); the flag is raised
// only by the one-lane kernel k_pass_latch launched after each pass's
// solves, so a launch sees the failures of earlier passes only.
__device__ __forceinline__ bool pass_halted(const unsigned long long *flags)
{
    return __hip_atomic_load(flags + kStopWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
}

}  // namespace tfk
