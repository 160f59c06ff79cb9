// Row-update kernels of one mode pass (eq. (SALS) and its B / c, arXiv:1410.5209).
//
// k_accum: for every row i of mode n (or one chunk of a long row), walk the
//   row's entries in the mode-n copy (CSR order), gather the other modes'
//   slab rows, form p_j = prod_{l != n} a^(l)_{i_l, S} and accumulate the Gram
//   matrix B = sum p p^T (upper triangle) and the right-hand side
//   c = sum rhat_j p_j.  G lanes share a row; each lane keeps a private partial
//   record in registers and the group sums them at the end.
//   In the first pass of a split (FIRST) the same walk also brings this copy of
//   the residual up to date: it subtracts the columns of the previous split
//   with their final values (eq. (SALS_R)) and adds the columns of this split
//   with their values at the start of the split (R-hat, Algorithm 1).
//   A factor row of a split lives in one interleaved slab row
//   [W: current | P: previous split, final | S: this split, at its start]
//   inside a 128-byte line, so every entry costs one line request per other
//   mode in every pass (random line requests, not bytes, bound this kernel).
// k_solve: one lane per row solves (B + lambda_i I) a = c in FP64 by
//   Cholesky (text after Theorem 1) and writes a into the mode's slab.
#pragma once

#include "dev_common.h"

namespace tfk {

// FM: 0 a plain pass; 1 a split's first pass in which no other mode has
// been updated yet (the split-start segments S equal W and are not read);
// 2 a first pass that reads S for the modes already updated.
template <int PREC, int CP, int NO, int FM>
__global__ __launch_bounds__(256) void k_accum(AccumArgs a)
{
    constexpr bool FIRST = FM > 0;
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    using TA = typename Types<PREC>::TA;
    constexpr int NE = gram_entries(CP);
    constexpr int NEP = gram_stride(CP);

    const int lane = threadIdx.x & 63;
    // a wavefront's task: by its place in the grid, or (persistent launch)
    // taken from the work counter until none is left (uniform per wavefront)
    int t = a.work ? take_task(a.work) : blockIdx.x * 4 + (threadIdx.x >> 6);
    for (; t < a.ntasks; t = take_task(a.work)) {
    const Task task = a.tasks[t];
    const int G = task.G;
    const int lg = __ffs(G) - 1;
    const int grp = lane >> lg;
    const int sub = lane & (G - 1);

    int row = -1;
    int64_t beg = 0, end = 0;
    TA *out = nullptr;
    if (task.kind == 0) {
        if (grp < task.count) {
            row = a.items[task.base + grp];
            beg = a.rowptr[row];
            end = a.rowptr[row + 1];
            out = reinterpret_cast<TA *>(a.gram) + (int64_t)row * NEP;
        }
    } else {
        const Chunk c = a.chunks[task.base];
        row = c.row;
        beg = c.beg;
        end = c.end;
        out = reinterpret_cast<TA *>(a.gpart) + (int64_t)c.slot * NEP;
    }

    const int64_t ld = a.ld;
    TR *rhat = reinterpret_cast<TR *>(a.rhat);

    TA own_p[CP], own_s[CP];
    if constexpr (FIRST) {
        if (row >= 0) {
            load_row<CP>(reinterpret_cast<const TS *>(a.Sown) + (int64_t)row * ld, own_s);
            if (a.has_pend)
                load_row8<CP>(reinterpret_cast<const TS *>(a.Pown) + (int64_t)row * ld, own_p);
            else {
#pragma unroll
                for (int c = 0; c < CP; ++c) own_p[c] = TA(0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < CP; ++c) { own_p[c] = TA(0); own_s[c] = TA(0); }
        }
    }

    TA acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = TA(0);

    int64_t j = beg + sub;
    if constexpr (!FIRST) {
        // Software pipeline: the factor rows of the next entry are requested
        // before the current entry is folded in, and the indices one entry
        // further ahead, so a lane keeps gathers in flight while it computes.
        // (with a.rperm the residual is read from another mode's copy)
        const int32_t *rperm = a.rperm;
        auto load_r = [&](int64_t jj) -> TR {
            return rperm ? stream_load(rhat + stream_load(rperm + jj)) : stream_load(rhat + jj);
        };
        int32_t ii[NO];
        TR rh = TR(0);
        TA w[NO][CP];
        if (j < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) ii[l] = stream_load(a.oidx[l] + j);
            rh = load_r(j);
#pragma unroll
            for (int l = 0; l < NO; ++l)
                load_row<CP>(reinterpret_cast<const TS *>(a.W[l]) + (int64_t)ii[l] * ld, w[l]);
        }
        int64_t jn = j + G;
        int32_t in_[NO];
        TR rn = TR(0);
        if (jn < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) in_[l] = stream_load(a.oidx[l] + jn);
            rn = load_r(jn);
        }
        while (j < end) {
            TA p[CP];
#pragma unroll
            for (int c = 0; c < CP; ++c) p[c] = w[0][c];
#pragma unroll
            for (int l = 1; l < NO; ++l)
#pragma unroll
                for (int c = 0; c < CP; ++c) p[c] *= w[l][c];
            const TA r = (TA)rh;
            if (jn < end) {
                rh = rn;
#pragma unroll
                for (int l = 0; l < NO; ++l)
                    load_row<CP>(reinterpret_cast<const TS *>(a.W[l]) + (int64_t)in_[l] * ld, w[l]);
                const int64_t jnn = jn + G;
                if (jnn < end) {
#pragma unroll
                    for (int l = 0; l < NO; ++l) in_[l] = stream_load(a.oidx[l] + jnn);
                    rn = load_r(jnn);
                }
            }
            int e = 0;
#pragma unroll
            for (int c1 = 0; c1 < CP; ++c1)
#pragma unroll
                for (int c2 = c1; c2 < CP; ++c2) acc[e++] += p[c1] * p[c2];
#pragma unroll
            for (int c = 0; c < CP; ++c) acc[e++] += r * p[c];
            j = jn;
            jn += G;
        }
    } else if constexpr (CP * NO <= 24) {
        // First pass of a split: the same pipeline, with each entry's three
        // segments (current W, previous split's final P, this split's start S
        // for modes already updated) requested one entry ahead.  Only for
        // small widths: three segments per other mode, twice, must stay in
        // registers.
        auto fetch = [&](const int32_t (&ix)[NO], TA (&w)[NO][CP], TA (&pv)[NO][CP],
                         TA (&sv)[NO][CP]) {
#pragma unroll
            for (int l = 0; l < NO; ++l) {
                const TS *row_l = reinterpret_cast<const TS *>(a.W[l]) + (int64_t)ix[l] * ld;
                load_row<CP>(row_l, w[l]);
                if (a.has_pend)
                    load_row8<CP>(reinterpret_cast<const TS *>(a.P[l]) + (int64_t)ix[l] * ld, pv[l]);
                if (FM == 2 && a.before[l])
                    load_row<CP>(reinterpret_cast<const TS *>(a.S[l]) + (int64_t)ix[l] * ld, sv[l]);
            }
        };
        int32_t ii[NO];
        TR rh = TR(0);
        TA w[NO][CP], pv[NO][CP], sv[NO][CP];
        if (j < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) ii[l] = stream_load(a.oidx[l] + j);
            rh = stream_load(rhat + j);
            fetch(ii, w, pv, sv);
        }
        int64_t jn = j + G;
        int32_t in_[NO];
        TR rn = TR(0);
        if (jn < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) in_[l] = stream_load(a.oidx[l] + jn);
            rn = stream_load(rhat + jn);
        }
        while (j < end) {
            TA p[CP], tp[CP], ts[CP];
#pragma unroll
            for (int c = 0; c < CP; ++c) { p[c] = w[0][c]; tp[c] = own_p[c]; ts[c] = own_s[c]; }
#pragma unroll
            for (int l = 1; l < NO; ++l)
#pragma unroll
                for (int c = 0; c < CP; ++c) p[c] *= w[l][c];
#pragma unroll
            for (int l = 0; l < NO; ++l) {
                if (a.has_pend) {
#pragma unroll
                    for (int c = 0; c < CP; ++c) tp[c] *= pv[l][c];
                }
                if (FM == 2 && a.before[l]) {
#pragma unroll
                    for (int c = 0; c < CP; ++c) ts[c] *= sv[l][c];
                } else {
#pragma unroll
                    for (int c = 0; c < CP; ++c) ts[c] *= w[l][c];
                }
            }
            const TR rcur = rh;
            const int64_t jcur = j;
            if (jn < end) {
                rh = rn;
                fetch(in_, w, pv, sv);
                const int64_t jnn = jn + G;
                if (jnn < end) {
#pragma unroll
                    for (int l = 0; l < NO; ++l) in_[l] = stream_load(a.oidx[l] + jnn);
                    rn = stream_load(rhat + jnn);
                }
            }
            // R-hat of this split from the previous split's residual state
            TA dr = TA(0), ds = TA(0);
#pragma unroll
            for (int c = 0; c < CP; ++c) { dr += tp[c]; ds += ts[c]; }
            const TA r = ((TA)rcur - dr) + ds;
            stream_store((TR)r, rhat + jcur);

            int e = 0;
#pragma unroll
            for (int c1 = 0; c1 < CP; ++c1)
#pragma unroll
                for (int c2 = c1; c2 < CP; ++c2) acc[e++] += p[c1] * p[c2];
#pragma unroll
            for (int c = 0; c < CP; ++c) acc[e++] += r * p[c];
            j = jn;
            jn += G;
        }
    } else {
        // First pass of a split, wider rows: indices and residual prefetched
        int32_t ii[NO];
        TR rh = TR(0);
        if (j < end) {
#pragma unroll
            for (int l = 0; l < NO; ++l) ii[l] = stream_load(a.oidx[l] + j);
            rh = stream_load(rhat + j);
        }
        for (; j < end; j += G) {
            int32_t cur[NO];
#pragma unroll
            for (int l = 0; l < NO; ++l) cur[l] = ii[l];
            TR rcur = rh;
            const int64_t jn = j + G;
            if (jn < end) {  // prefetch the next entry's indices and residual
#pragma unroll
                for (int l = 0; l < NO; ++l) ii[l] = stream_load(a.oidx[l] + jn);
                rh = stream_load(rhat + jn);
            }
            TA w[NO][CP];
#pragma unroll
            for (int l = 0; l < NO; ++l)
                load_row<CP>(reinterpret_cast<const TS *>(a.W[l]) + (int64_t)cur[l] * ld, w[l]);
            TA p[CP];
#pragma unroll
            for (int c = 0; c < CP; ++c) p[c] = w[0][c];
#pragma unroll
            for (int l = 1; l < NO; ++l)
#pragma unroll
                for (int c = 0; c < CP; ++c) p[c] *= w[l][c];

            // R-hat of this split from the previous split's residual state
            TA tp[CP], ts[CP];
#pragma unroll
            for (int c = 0; c < CP; ++c) { tp[c] = own_p[c]; ts[c] = own_s[c]; }
#pragma unroll
            for (int l = 0; l < NO; ++l) {
                if (a.has_pend) {
                    TA v[CP];
                    load_row8<CP>(reinterpret_cast<const TS *>(a.P[l]) + (int64_t)cur[l] * ld, v);
#pragma unroll
                    for (int c = 0; c < CP; ++c) tp[c] *= v[c];
                }
                if (FM == 2 && a.before[l]) {
                    TA v[CP];
                    load_row<CP>(reinterpret_cast<const TS *>(a.S[l]) + (int64_t)cur[l] * ld, v);
#pragma unroll
                    for (int c = 0; c < CP; ++c) ts[c] *= v[c];
                } else {
#pragma unroll
                    for (int c = 0; c < CP; ++c) ts[c] *= w[l][c];
                }
            }
            TA dr = TA(0), ds = TA(0);
#pragma unroll
            for (int c = 0; c < CP; ++c) { dr += tp[c]; ds += ts[c]; }
            const TA r = ((TA)rcur - dr) + ds;
            stream_store((TR)r, rhat + j);

            int e = 0;
#pragma unroll
            for (int c1 = 0; c1 < CP; ++c1)
#pragma unroll
                for (int c2 = c1; c2 < CP; ++c2) acc[e++] += p[c1] * p[c2];
#pragma unroll
            for (int c = 0; c < CP; ++c) acc[e++] += r * p[c];
        }
    }

    group_reduce<NE>(acc, G);

    if (row >= 0 && sub == 0) {
        if constexpr (sizeof(TA) == 4) {
            float4 *o = reinterpret_cast<float4 *>(out);
#pragma unroll
            for (int v = 0; v < NEP / 4; ++v) {
                float4 q;
                q.x = 4 * v + 0 < NE ? acc[4 * v + 0] : 0.f;
                q.y = 4 * v + 1 < NE ? acc[4 * v + 1] : 0.f;
                q.z = 4 * v + 2 < NE ? acc[4 * v + 2] : 0.f;
                q.w = 4 * v + 3 < NE ? acc[4 * v + 3] : 0.f;
                o[v] = q;
            }
        } else {
            double2 *o = reinterpret_cast<double2 *>(out);
#pragma unroll
            for (int v = 0; v < NEP / 2; ++v) {
                double2 q;
                q.x = 2 * v + 0 < NE ? acc[2 * v + 0] : 0.0;
                q.y = 2 * v + 1 < NE ? acc[2 * v + 1] : 0.0;
                o[v] = q;
            }
        }
    }
    if (!a.work) break;
    }
}

// Index of B(c1, c2), c1 <= c2, in the packed upper-triangle record.
__host__ __device__ constexpr int upper_index(int CP, int c1, int c2)
{
    return c1 * CP - c1 * (c1 - 1) / 2 + (c2 - c1);
}

// Solve of one row: (B + lambda_i I) a = c from its Gram record g, written
// to o in the storage type; false (and nothing written) for a non-positive
// pivot.
template <int PREC, int CP>
__device__ __forceinline__ bool solve_row(const typename Types<PREC>::TA *g, double lam,
                                          typename Types<PREC>::TS *o)
{
    using TS = typename Types<PREC>::TS;
    constexpr int NT = CP * (CP + 1) / 2;
    double L[NT];   // packed lower triangle, L(i, k) at i*(i+1)/2 + k
    double y[CP];
#pragma unroll
    for (int i = 0; i < CP; ++i) {
#pragma unroll
        for (int k = 0; k <= i; ++k) L[i * (i + 1) / 2 + k] = (double)g[upper_index(CP, k, i)];
        L[i * (i + 1) / 2 + i] += lam;
        y[i] = (double)g[NT + i];
    }
    bool ok = true;
#pragma unroll
    for (int jj = 0; jj < CP; ++jj) {
        double d = L[jj * (jj + 1) / 2 + jj];
#pragma unroll
        for (int k = 0; k < jj; ++k) d -= L[jj * (jj + 1) / 2 + k] * L[jj * (jj + 1) / 2 + k];
        ok = ok && (d > 0.0);
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        L[jj * (jj + 1) / 2 + jj] = ljj;
#pragma unroll
        for (int i = jj + 1; i < CP; ++i) {
            double s = L[i * (i + 1) / 2 + jj];
#pragma unroll
            for (int k = 0; k < jj; ++k) s -= L[i * (i + 1) / 2 + k] * L[jj * (jj + 1) / 2 + k];
            L[i * (i + 1) / 2 + jj] = s / ljj;
        }
    }
    if (!ok) return false;
#pragma unroll
    for (int i = 0; i < CP; ++i) {
        double s = y[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i * (i + 1) / 2 + k] * y[k];
        y[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = CP - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < CP; ++k) s -= L[k * (k + 1) / 2 + i] * y[k];
        y[i] = s / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int c = 0; c < CP; ++c) o[c] = store_cast<TS>(y[c]);
    return true;
}

template <int PREC, int CP>
__global__ __launch_bounds__(256) void k_solve(SolveArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TA = typename Types<PREC>::TA;
    constexpr int NEP = gram_stride(CP);
    if (pass_halted(a.flags)) return;   // uniform: no factor changes after a failed pass

    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row < a.I) {
        const int64_t cnt = (int64_t)a.rowptr[row + 1] - a.rowptr[row];
        TS *o = reinterpret_cast<TS *>(a.W) + row * a.ld;
        if (cnt == 0) {  // a row with no observed entries is set to zero
#pragma unroll
            for (int c = 0; c < CP; ++c) o[c] = store_cast<TS>(0.0);
        } else {
            const TA *g = reinterpret_cast<const TA *>(a.gram) + row * NEP;
            const double lam = a.reg_mode ? a.lambda * (double)cnt : a.lambda;
            if (!solve_row<PREC, CP>(g, lam, o)) atomicMin(a.bad, (unsigned long long)row);
        }
    }
}

// Sum of the chunk partials of each split row into the row's Gram record.
// Every thread owns some entries of the record; chunk c goes to partial sum
// c mod 8, and the eight partials are added in a fixed tree, so the result
// does not depend on scheduling (and eight loads are in flight per thread).
template <int PREC, int CP>
__global__ __launch_bounds__(256) void k_chunk_reduce(const int32_t *split_rows,
                                                      const int32_t *ptr, const void *gpart,
                                                      void *gram)
{
    using TA = typename Types<PREC>::TA;
    constexpr int NE = gram_entries(CP);
    constexpr int NEP = gram_stride(CP);
    const int b = blockIdx.x;
    const int row = split_rows[b];
    const TA *gp = reinterpret_cast<const TA *>(gpart);
    TA *gr = reinterpret_cast<TA *>(gram) + (int64_t)row * NEP;
    const int c0 = ptr[b], c1 = ptr[b + 1];
    for (int e = threadIdx.x; e < NEP; e += blockDim.x) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (e < NE) {
            int c = c0;
            for (; c + 8 <= c1; c += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) s[u] += (double)gp[(int64_t)(c + u) * NEP + e];
            }
            for (int u = 0; c < c1; ++c, ++u) s[u] += (double)gp[(int64_t)c * NEP + e];
        }
        gr[e] = (TA)(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
    }
}

}  // namespace tfk
