// Row-update kernels for splits of 32 columns (eq. (SALS) and its B / c,
// arXiv:1410.5209), FP32 or BF16 storage.
//
// k_accum_wide: one wavefront walks a row (or a chunk of one) two entries at
//   a time: lane 32h + c holds column c of the step's entry h, so each half
//   wavefront reads whole 128-byte factor rows with one coalesced load per
//   mode.  The lane forms its column of p_j = prod_{l != n} a^(l) (and, in a
//   split's first pass, its column of the residual update, summed over the
//   half).  B = sum_j p_j p_j^T is a dense contraction over the row's
//   entries: one v_mfma_f32_32x32x2f32 per step adds both entries' outer
//   products to the 32x32 FP32 accumulator; c = sum_j rhat_j p_j stays on
//   the vector unit.  Entry indices and residuals are staged 64 at a time
//   (one per lane) and passed to the halves by lane permutes; first-pass
//   residuals are written back 64 at a time.
// k_solve_wide: half a wavefront per row: (B + lambda_i I) a = c in FP64 by
//   Cholesky (text after Theorem 1), M = L L^T computed in place with lane i
//   holding row i of the lower triangle in registers.  Step j: lane j forms
//   1 / L(j, j) and y_j, which reach the half by lane reads; lanes i > j form
//   L(i, j) and store it as column j of L in LDS, from where every lane
//   updates its row.  Back substitution L^T a = y: lane i takes column i of L
//   from LDS, and each a_k reaches the half by lane reads.  a goes to the W
//   segment of the mode's slab.
#pragma once

#include "dev_common.h"

namespace tfk {

constexpr int WCP = 32;                       // columns per split
constexpr int WNT = WCP * (WCP + 1) / 2;      // 528 Gram entries (upper)

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Column c of a factor-row segment, in two steps so that a group's loads
// are all issued before any result is used: load_raw fetches the 4-byte word
// holding the column (BF16: the lane pair 2k, 2k+1 shares one word),
// col_value turns it into the column's FP32 value.
__device__ __forceinline__ uint32_t load_raw(const float *row, int c)
{
    return __float_as_uint(row[c]);
}
__device__ __forceinline__ uint32_t load_raw(const bf16 *row, int c)
{
    return reinterpret_cast<const uint32_t *>(row)[c >> 1];
}
template <typename TS> __device__ __forceinline__ float col_value(uint32_t x, int c);
template <> __device__ __forceinline__ float col_value<float>(uint32_t x, int) { return __uint_as_float(x); }
template <> __device__ __forceinline__ float col_value<bf16>(uint32_t x, int c)
{
    return __uint_as_float((c & 1) ? (x & 0xffff0000u) : (x << 16));
}
template <typename TS> __device__ __forceinline__ float load_col(const TS *row, int c)
{
    return col_value<TS>(load_raw(row, c), c);
}

// Sum over each 32-lane half: quad swaps, half-row and row mirrors, then the
// two rows of the half.
__device__ __forceinline__ float half_sum(float v)
{
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += __shfl_xor(v, 16, 64);
    return v;
}

// FM: 0 a plain pass, 1 a split's first pass with no other mode updated yet
// in the split (no split-start segments to read: they equal W), 2 a first
// pass that reads them for the modes already updated.
template <int PREC, int NO, int FM>
__global__ __launch_bounds__(256) void k_accum_wide(AccumArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    static_assert(sizeof(typename Types<PREC>::TA) == 4, "wide kernel accumulates in FP32");
    constexpr int NEP = gram_stride(WCP);
    constexpr int GS = 4;                        // steps whose loads are issued together
    constexpr bool FIRST = FM > 0;

    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int c = lane & 31;
    // a wavefront's task: by its place in the grid, or (persistent launch)
    // taken from the work counter until none is left (uniform per
    // wavefront; no block barriers below)
    int t = a.work ? take_task(a.work) : blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ld = a.ld;
    TR *rhat = reinterpret_cast<TR *>(a.rhat);
    for (; t < a.ntasks; t = take_task(a.work)) {
    const Task task = a.tasks[t];

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
            const Chunk ch = a.chunks[task.base];
            row = ch.row;
            beg = ch.beg;
            end = ch.end;
            out = reinterpret_cast<float *>(a.gpart) + (int64_t)ch.slot * NEP;
        }
        float own_p = 0.f, own_s = 0.f;
        if constexpr (FIRST) {
            own_s = load_col(reinterpret_cast<const TS *>(a.Sown) + (int64_t)row * ld, c);
            if (a.has_pend) own_p = load_col(reinterpret_cast<const TS *>(a.Pown) + (int64_t)row * ld, c);
        }
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
        float rhs = 0.f;

        for (int64_t s0 = beg; s0 < end; s0 += 64) {
            // stage 64 entries: lane L holds entry s0 + L
            const int64_t jl = s0 + lane;
            const bool lv = jl < end;
            int32_t bidx[NO];
#pragma unroll
            for (int l = 0; l < NO; ++l) bidx[l] = lv ? stream_load(a.oidx[l] + jl) : 0;
            // residuals read through another mode's order are used once: a
            // streaming load keeps their lines from displacing factor rows in L2
            float brh = 0.f;
            if (lv) brh = (float)(a.rperm ? stream_load(rhat + stream_load(a.rperm + jl)) : stream_load(rhat + jl));
            float rnew = 0.f;
            const int nstep = (int)((end - s0 + 1) / 2 < 32 ? (end - s0 + 1) / 2 : 32);
            for (int u0 = 0; u0 < nstep; u0 += GS) {
                uint32_t w[GS][NO], pv[GS][NO], sv[GS][NO];
                float rq[GS];
                bool val[GS];
#pragma unroll
                for (int q = 0; q < GS; ++q) {
                    const int src = (2 * (u0 + q) + half) & 63;
                    val[q] = u0 + q < nstep && s0 + src < end;
                    int32_t ii[NO];
#pragma unroll
                    for (int l = 0; l < NO; ++l) ii[l] = __shfl(bidx[l], src, 64);
                    rq[q] = __shfl(brh, src, 64);
#pragma unroll
                    for (int l = 0; l < NO; ++l) {
                        w[q][l] = pv[q][l] = sv[q][l] = 0u;
                        if (val[q]) {
                            const int64_t off = (int64_t)ii[l] * ld;
                            w[q][l] = load_raw(reinterpret_cast<const TS *>(a.W[l]) + off, c);
                            if constexpr (FIRST) {
                                if (a.has_pend) pv[q][l] = load_raw(reinterpret_cast<const TS *>(a.P[l]) + off, c);
                                if (FM == 2 && a.before[l]) sv[q][l] = load_raw(reinterpret_cast<const TS *>(a.S[l]) + off, c);
                            }
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < GS; ++q) {
                    float wv[NO];
#pragma unroll
                    for (int l = 0; l < NO; ++l) wv[l] = col_value<TS>(w[q][l], c);
                    float p = val[q] ? wv[0] : 0.f;
#pragma unroll
                    for (int l = 1; l < NO; ++l) p *= wv[l];
                    float r = rq[q];
                    if constexpr (FIRST) {
                        // R-hat of this split: the previous split's columns
                        // (final values) out, this split's (start values) in
                        float tp = val[q] ? own_p : 0.f, ts = val[q] ? own_s : 0.f;
#pragma unroll
                        for (int l = 0; l < NO; ++l) {
                            tp *= col_value<TS>(pv[q][l], c);
                            ts *= (FM == 2 && a.before[l]) ? col_value<TS>(sv[q][l], c) : wv[l];
                        }
                        r = (r - half_sum(tp)) + half_sum(ts);
                        const float rh0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r), 0));
                        const float rh1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r), 32));
                        const int u = u0 + q;
                        if (lane == 2 * u) rnew = rh0;
                        if (lane == 2 * u + 1) rnew = rh1;
                    }
                    if (!val[q]) r = 0.f;
                    rhs += r * p;
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(p, p, acc, 0, 0, 0);
                }
            }
            if constexpr (FIRST) {
                if (lv) stream_store((TR)rnew, rhat + jl);
            }
        }
        rhs += __shfl_xor(rhs, 32, 64);
        // Gram record: upper triangle of B, then c.  Accumulator register r
        // of lane 32h + c holds B(8 (r / 4) + 4 h + r % 4, c).
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r / 4) + 4 * half + (r % 4);
            if (i <= c) out[i * WCP - i * (i - 1) / 2 + (c - i)] = acc[r];
        }
        if (half == 0) out[WNT + c] = rhs;
        if (lane < NEP - WNT - WCP) out[WNT + WCP + lane] = 0.f;
    }
    if (!a.work) break;
    }
}

// A double from lane k of each 32-lane half, returned to every lane of that
// half (k is a compile-time lane number in the callers).
__device__ __forceinline__ double half_bcast(double v, int k, int half)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo0 = __builtin_amdgcn_readlane(lo, k), hi0 = __builtin_amdgcn_readlane(hi, k);
    const int lo1 = __builtin_amdgcn_readlane(lo, k + 32), hi1 = __builtin_amdgcn_readlane(hi, k + 32);
    return half ? __hiloint2double(hi1, lo1) : __hiloint2double(hi0, lo0);
}

// 1 / sqrt(d) for d > 0: hardware estimate, then two steps of Newton's
// iteration r <- r (3 - d r^2) / 2 (each roughly doubles the correct bits).
__device__ __forceinline__ double rsqrt_nr(double d)
{
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}

template <int PREC>
__global__ __launch_bounds__(256) void k_solve_wide(SolveArgs a)
{
    using TS = typename Types<PREC>::TS;
    constexpr int NEP = gram_stride(WCP);
    constexpr int NV = NEP / 4;
    constexpr int LT = WCP * (WCP - 1) / 2;     // strictly lower entries of L
    static_assert(NEP * sizeof(float) <= LT * sizeof(double), "record must fit the L area");
    // per row: first the staged Gram record, then the columns of L below the
    // diagonal (column j at colofs(j), rows j+1..31)
    __shared__ __align__(16) double lt[8][LT];
    if (pass_halted(a.flags)) return;   // uniform: no factor changes after a failed pass
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int i = lane & 31;
    const int slot = 2 * wave + half;
    const int64_t row0 = (int64_t)blockIdx.x * 8 + 2 * wave;
    const int64_t row = row0 + half;
    auto colofs = [](int j) { return j * (WCP - 1) - j * (j - 1) / 2; };

    // the wavefront's two records, coalesced, into LDS
    const float4 *gsrc = reinterpret_cast<const float4 *>(a.gram);
    for (int v = lane; v < 2 * NV; v += 64) {
        const int r = v >= NV ? 1 : 0;
        const int q = v - r * NV;
        if (row0 + r < a.I)
            reinterpret_cast<float4 *>(lt[2 * wave + r])[q] = gsrc[(row0 + r) * NV + q];
    }
    __builtin_amdgcn_wave_barrier();

    const bool valid = row < a.I;
    const int64_t cnt = valid ? (int64_t)a.rowptr[row + 1] - a.rowptr[row] : 0;
    const bool live = cnt > 0;
    const float *rf = reinterpret_cast<const float *>(lt[slot]);
    // lane i: M(i, k) for k <= i, which is record entry (k, i) of the upper
    // triangle, and c_i; an empty or absent row solves the identity system.
    // Slots k > i are scratch until the back substitution, where they hold
    // column i of L.
    const double lam = a.reg_mode ? a.lambda * (double)cnt : a.lambda;
    double m[WCP];
#pragma unroll
    for (int k = 0; k < WCP; ++k) {
        const int idx = k * WCP - k * (k - 1) / 2 - k + i;
        m[k] = (live && k <= i) ? (double)rf[idx] : 0.0;
        if (k == i) m[k] = live ? m[k] + lam : 1.0;
    }
    double c = live ? (double)rf[WNT + i] : 0.0;
    // the record is consumed before L overwrites it
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();

    double *L = lt[slot];
    bool ok = true;
    double rinv = 1.0;
#pragma unroll
    for (int j = 0; j < WCP; ++j) {
        if (i == j) {
            const double d = m[j];
            ok = d > 0.0;
            const double dd = ok ? d : 1.0;
            rinv = rsqrt_nr(dd);        // 1 / L(j, j)
            m[j] = dd * rinv;
            c *= rinv;                  // y_j of L y = c
        }
        const double dj = half_bcast(rinv, j, half), yj = half_bcast(c, j, half);
        double lij = 0.0;
        if (i > j) {
            lij = m[j] * dj;            // L(i, j)
            m[j] = lij;
            c -= lij * yj;
            L[colofs(j) + i - j - 1] = lij;
        }
        __builtin_amdgcn_wave_barrier();
        // M(i, k) -= L(i, j) L(k, j); lanes i <= j have lij = 0 and only
        // scratch slots at k > j.  The column is read eight values at a time
        // (the memory clobber keeps later groups' reads from being hoisted)
        // and each update is pinned to this step by an empty asm (left to
        // itself the compiler defers the updates and keeps columns of
        // several steps live in registers).
#pragma unroll
        for (int k0 = j + 1; k0 < WCP; k0 += 8) {
            double col[8];
#pragma unroll
            for (int k = k0; k < k0 + 8 && k < WCP; ++k) col[k - k0] = L[colofs(j) + k - j - 1];
#pragma unroll
            for (int k = k0; k < k0 + 8 && k < WCP; ++k) {
                m[k] -= lij * col[k - k0];
                asm volatile("" : "+v"(m[k]));
            }
            asm volatile("" ::: "memory");
        }
    }
    __builtin_amdgcn_wave_barrier();
    // column i of L into the scratch slots, then L^T a = y, last unknown first
    const int ci = colofs(i) - i - 1;
#pragma unroll
    for (int k = 1; k < WCP; ++k)
        if (k > i) m[k] = L[ci + k];
#pragma unroll
    for (int k = WCP - 1; k >= 0; --k) {
        if (i == k) c *= rinv;          // a_k
        const double ak = half_bcast(c, k, half);
        if (i < k) c -= m[k] * ak;
    }

    const unsigned long long bad = __ballot(!ok);
    const bool row_bad = ((bad >> (32 * half)) & 0xffffffffull) != 0ull;
    if (valid) {
        TS *o = reinterpret_cast<TS *>(a.W) + row * a.ld;
        if (!live) o[i] = store_cast<TS>(0.0);
        else if (row_bad) {
            if (i == 0) atomicMin(a.bad, (unsigned long long)row);
        } else {
            o[i] = store_cast<TS>(c);
        }
    }
}

}  // namespace tfk
