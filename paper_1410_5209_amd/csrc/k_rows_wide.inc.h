// Row-update kernels for splits of 32 columns (eq. (SALS) and its B / c,
// arXiv:1410.5209), FP32 or BF16 storage.
//
// k_accum_wide: one wavefront walks a row (or a chunk of one) eight entries at
//   a time.  Gather phase: lane 8e+q holds columns 4q..4q+3 of entry e, so one
//   16-byte load per lane fetches eight whole 128-byte factor rows per
//   instruction; the lane forms its four columns of p_j = prod_{l != n} a^(l)
//   and, in a split's first pass, its share of the residual update (summed
//   over the entry's eight lanes).  The eight p vectors go to LDS.
//   Accumulate phase: lane (bi, bj) owns the 4x4 block (rows 4bi.., columns
//   4bj..) of B = sum p p^T and, for bj = 0, four entries of c = sum rhat p;
//   each staged entry is a rank-1 update of that block from two 16-byte LDS
//   reads.  No cross-lane reduction is needed at the end of a row.
// k_solve_wide: one wavefront per row: (B + lambda_i I) a = c in FP64 by a
//   column Cholesky in LDS (text after Theorem 1), then the two triangular
//   solves; a goes to the W segment of the mode's slab.
#pragma once

#include "dev_common.h"

namespace tfk {

constexpr int WCP = 32;                       // columns per split
constexpr int WNT = WCP * (WCP + 1) / 2;      // 528 Gram entries (upper)

// Four consecutive storage elements -> float (16-byte or 8-byte load).
__device__ __forceinline__ void load4(const float *__restrict__ p, float (&o)[4])
{
    const float4 t = *reinterpret_cast<const float4 *>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
}
__device__ __forceinline__ void load4(const bf16 *__restrict__ p, float (&o)[4])
{
    const uint2 t = *reinterpret_cast<const uint2 *>(p);
    o[0] = __uint_as_float(t.x << 16); o[1] = __uint_as_float(t.x & 0xffff0000u);
    o[2] = __uint_as_float(t.y << 16); o[3] = __uint_as_float(t.y & 0xffff0000u);
}

// Sum over the eight lanes of an entry (lanes 8e..8e+7): xor 1, xor 2, then
// the half-row mirror pairs the two quads.
__device__ __forceinline__ float sum8(float v)
{
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    return v;
}

template <int PREC, int NO, bool FIRST>
__global__ __launch_bounds__(256) void k_accum_wide(AccumArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    static_assert(sizeof(typename Types<PREC>::TA) == 4, "wide kernel accumulates in FP32");
    constexpr int NEP = gram_stride(WCP);
    __shared__ float4 lds_p[4][8][WCP / 4];     // per wave: 8 staged p vectors
    __shared__ float lds_r[4][8];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 4 + wave;
    if (t >= a.ntasks) return;  // uniform per wavefront; no block barriers below
    const Task task = a.tasks[t];
    const int64_t ld = a.ld;
    TR *rhat = reinterpret_cast<TR *>(a.rhat);

    const int e = lane >> 3;        // gather phase: entry slot
    const int q = lane & 7;         // gather phase: column quad
    const int bi = lane >> 3;       // accumulate phase: block row
    const int bj = lane & 7;        // accumulate phase: block column

    const int nrows = task.kind == 0 ? task.count : 1;
    for (int rr = 0; rr < nrows; ++rr) {
        int row;
        int64_t beg, end;
        float *out;
        if (task.kind == 0) {
            row = a.items[task.base + rr];
            beg = a.rowptr[row];
            end = a.rowptr[row + 1];
            out = reinterpret_cast<float *>(a.gram) + (int64_t)row * NEP;
        } else {
            const Chunk c = a.chunks[task.base];
            row = c.row;
            beg = c.beg;
            end = c.end;
            out = reinterpret_cast<float *>(a.gpart) + (int64_t)c.slot * NEP;
        }
        float own_p[4], own_s[4];
        if constexpr (FIRST) {
            load4(reinterpret_cast<const TS *>(a.Sown) + (int64_t)row * ld + 4 * q, own_s);
            if (a.has_pend) load4(reinterpret_cast<const TS *>(a.Pown) + (int64_t)row * ld + 4 * q, own_p);
            else { own_p[0] = own_p[1] = own_p[2] = own_p[3] = 0.f; }
        }
        float acc[4][4], rhs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rhs[u] = 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.f;
        }
        // indices and residual of the next step are requested while the
        // current step's factor rows are gathered and folded in
        int32_t nx[NO];
        TR nr = TR(0);
        if (beg + e < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) nx[l] = a.oidx[l][beg + e];
            nr = rhat[beg + e];
        }
        for (int64_t s0 = beg; s0 < end; s0 += 8) {
            const int64_t j = s0 + e;
            const bool valid = j < end;
            int32_t ii[NO];
#pragma unroll
            for (int l = 0; l < NO; ++l) ii[l] = nx[l];
            const TR rcur = nr;
            if (j + 8 < end) {
#pragma unroll
                for (int l = 0; l < NO; ++l) nx[l] = a.oidx[l][j + 8];
                nr = rhat[j + 8];
            }
            float p[4] = {0.f, 0.f, 0.f, 0.f};
            float r = 0.f, dr = 0.f, ds = 0.f;   // this lane's four columns of the update
            if (valid) {
                r = (float)rcur;
                float w[NO][4];
#pragma unroll
                for (int l = 0; l < NO; ++l)
                    load4(reinterpret_cast<const TS *>(a.W[l]) + (int64_t)ii[l] * ld + 4 * q, w[l]);
#pragma unroll
                for (int c = 0; c < 4; ++c) p[c] = w[0][c];
#pragma unroll
                for (int l = 1; l < NO; ++l)
#pragma unroll
                    for (int c = 0; c < 4; ++c) p[c] *= w[l][c];
                if constexpr (FIRST) {
                    float tp[4], ts[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) { tp[c] = own_p[c]; ts[c] = own_s[c]; }
#pragma unroll
                    for (int l = 0; l < NO; ++l) {
                        if (a.has_pend) {
                            float v[4];
                            load4(reinterpret_cast<const TS *>(a.P[l]) + (int64_t)ii[l] * ld + 4 * q, v);
#pragma unroll
                            for (int c = 0; c < 4; ++c) tp[c] *= v[c];
                        }
                        if (a.before[l]) {
                            float v[4];
                            load4(reinterpret_cast<const TS *>(a.S[l]) + (int64_t)ii[l] * ld + 4 * q, v);
#pragma unroll
                            for (int c = 0; c < 4; ++c) ts[c] *= v[c];
                        } else {
#pragma unroll
                            for (int c = 0; c < 4; ++c) ts[c] *= w[l][c];
                        }
                    }
                    dr = (tp[0] + tp[1]) + (tp[2] + tp[3]);
                    ds = (ts[0] + ts[1]) + (ts[2] + ts[3]);
                }
            }
            if constexpr (FIRST) {
                // R-hat of this split: subtract the previous split's columns
                // (final values), add this split's (start values); the sums
                // over the 32 columns run over the entry's eight lanes
                dr = sum8(dr);
                ds = sum8(ds);
                r = (r - dr) + ds;
                if (valid && q == 0) rhat[j] = (TR)r;
            }
            lds_p[wave][e][q] = make_float4(p[0], p[1], p[2], p[3]);
            if (q == 0) lds_r[wave][e] = valid ? r : 0.f;
            __builtin_amdgcn_wave_barrier();
            // accumulate phase: rank-1 updates of this lane's 4x4 block
#pragma unroll
            for (int ee = 0; ee < 8; ++ee) {
                const float4 x = lds_p[wave][ee][bi];
                const float4 y = lds_p[wave][ee][bj];
                const float xs[4] = {x.x, x.y, x.z, x.w};
                const float ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += xs[u] * ys[v];
                if (bj == 0) {
                    const float rr2 = lds_r[wave][ee];
#pragma unroll
                    for (int u = 0; u < 4; ++u) rhs[u] += rr2 * xs[u];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // Gram record: upper triangle of B, then c
        if (bi <= bj) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c1 = 4 * bi + u, c2 = 4 * bj + v;
                    if (c1 <= c2) out[c1 * WCP - c1 * (c1 - 1) / 2 + (c2 - c1)] = acc[u][v];
                }
        }
        if (bj == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) out[WNT + 4 * bi + u] = rhs[u];
        }
        if (lane < NEP - WNT - WCP) out[WNT + WCP + lane] = 0.f;
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_solve_wide(SolveArgs a)
{
    using TS = typename Types<PREC>::TS;
    constexpr int NEP = gram_stride(WCP);
    __shared__ double Ls[4][WNT];
    __shared__ double ys[4][WCP];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * 4 + wave;
    if (row >= a.I) return;
    const int64_t cnt = (int64_t)a.rowptr[row + 1] - a.rowptr[row];
    TS *o = reinterpret_cast<TS *>(a.W) + row * a.ld;
    if (cnt == 0) {
        if (lane < WCP) o[lane] = store_cast<TS>(0.0);
        return;
    }
    double *L = Ls[wave];
    double *y = ys[wave];
    const float *g = reinterpret_cast<const float *>(a.gram) + row * NEP;
    // upper record (c1 <= c2) -> packed lower L(c2, c1)
    for (int c1 = 0; c1 < WCP; ++c1) {
        const int len = WCP - c1;
        const int base = c1 * WCP - c1 * (c1 - 1) / 2;
        for (int d = lane; d < len; d += 64) {
            const int c2 = c1 + d;
            L[c2 * (c2 + 1) / 2 + c1] = (double)g[base + d];
        }
    }
    const double lam = a.reg_mode ? a.lambda * (double)cnt : a.lambda;
    if (lane < WCP) {
        y[lane] = (double)g[WNT + lane];
        L[lane * (lane + 1) / 2 + lane] += lam;
    }
    __builtin_amdgcn_wave_barrier();
    bool ok = true;
    for (int j = 0; j < WCP; ++j) {
        const double d = L[j * (j + 1) / 2 + j];
        ok = ok && d > 0.0;
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        __builtin_amdgcn_wave_barrier();
        if (lane == j) L[j * (j + 1) / 2 + j] = ljj;
        if (lane > j && lane < WCP) L[lane * (lane + 1) / 2 + j] /= ljj;
        __builtin_amdgcn_wave_barrier();
        // trailing update, pairs (i, k) with j < k <= i < WCP
        const int n = WCP - 1 - j;
        const int T = n * (n + 1) / 2;
        for (int pp = lane; pp < T; pp += 64) {
            int r = (int)((sqrtf(8.0f * (float)pp + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= pp) ++r;
            while (r * (r + 1) / 2 > pp) --r;
            const int i = j + 1 + r, k = j + 1 + (pp - r * (r + 1) / 2);
            L[i * (i + 1) / 2 + k] -= L[i * (i + 1) / 2 + j] * L[k * (k + 1) / 2 + j];
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!ok) {
        if (lane == 0) atomicMin(a.bad, (unsigned long long)row);
        return;
    }
    for (int k = 0; k < WCP; ++k) {          // L y = c
        const double yk = y[k] / L[k * (k + 1) / 2 + k];
        __builtin_amdgcn_wave_barrier();
        if (lane == k) y[k] = yk;
        if (lane > k && lane < WCP) y[lane] -= L[lane * (lane + 1) / 2 + k] * yk;
        __builtin_amdgcn_wave_barrier();
    }
    for (int k = WCP - 1; k >= 0; --k) {     // L^T a = y
        const double ak = y[k] / L[k * (k + 1) / 2 + k];
        __builtin_amdgcn_wave_barrier();
        if (lane == k) y[k] = ak;
        if (lane < k) y[lane] -= L[k * (k + 1) / 2 + lane] * ak;
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < WCP) o[lane] = store_cast<TS>(y[lane]);
}

}  // namespace tfk
