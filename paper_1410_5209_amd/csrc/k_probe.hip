// Measurement probe (not part of the method): the rate at which the GPU
// serves random 128-byte row gathers from a table of a given size.  The row
// passes of a split are bound by such requests (one line per gathered factor
// row), so this rate is the ceiling their line-request rate is compared with.
//
// Each half-wavefront reads one whole 128-byte row per step (32 lanes x 4
// bytes, one coalesced request), rows chosen by a counter-based hash (one
// draw per lane for 64 rows), so the probe reads no index stream.  Every
// lane keeps a running sum of what it read and writes it once, so no load
// can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tf.h"

namespace {

__device__ __forceinline__ uint64_t probe_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_probe_gather(const float *table, int64_t rows,
                                                      int64_t steps, uint64_t seed, float *out)
{
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int c = lane & 31;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    float acc = 0.f;
    constexpr int G = 8;   // rows requested together per half-wavefront
    // 64 rows per round (2 per step, 32 steps): lane L draws the row of step
    // L / 2, half L % 2, and the halves take them by lane permutes, as the
    // row kernels take their staged entry indices
    for (int64_t s0 = 0; s0 < 2 * steps; s0 += 64) {
        const uint64_t h = probe_mix(seed + (uint64_t)(wave * 2 * steps + s0 + lane) * 0x9E3779B97F4A7C15ull);
        const int64_t mine = (int64_t)(((h >> 32) * (uint64_t)rows) >> 32);   // in [0, rows)
        for (int u0 = 0; u0 < 32; u0 += G) {
            float v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int src = 2 * (u0 + g) + half;
                const int64_t r = __shfl(mine, src, 64);
                v[g] = table[r * 32 + c];
            }
#pragma unroll
            for (int g = 0; g < G; ++g) acc += v[g];
        }
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

extern "C" tf_status tf_probe_gather(const void *d_table, int64_t rows, int64_t waves,
                                     int64_t steps, uint64_t seed, float *d_out, void *stream,
                                     double *ms)
{
    if (!d_table || !d_out || !ms || rows < 1 || rows > ((int64_t)1 << 32) || waves < 4 ||
        waves % 4 != 0 || steps < 32 || steps % 32 != 0)
        return TF_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return TF_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TF_E_DEVICE;
    }
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_gather, dim3((unsigned)(waves / 4)), dim3(256), 0, st,
                           static_cast<const float *>(d_table), rows, steps, seed, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return TF_E_DEVICE;
    *ms = f;
    return TF_OK;
}
