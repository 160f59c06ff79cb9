// Row updates for splits wider than the register and wide kernels take
// (33..128 columns in FP32 / BF16 storage, 17..128 in FP64): eq. (SALS) with
// B and c defined beside it (arXiv:1410.5209), one workgroup per row, up to
// C = K, where the split is the ALS row solve of eq. (ALS).
//
// At these widths a row's C x C system no longer fits one lane or half a
// wavefront, so the path is built differently from the narrow kernels:
//  * R-hat is formed once per split on mode 1's residual copy by a separate
//    pass (k_big_boundary), and every mode reads that copy (through the
//    position map for modes 2..N): no split-start or pending segments.
//  * Factor rows are read and written in place in the factor matrices (the
//    split's columns through a column list), so no slabs are packed.
//  * k_big_rows: one 256-thread workgroup per row.  The row's entries are
//    staged 32 at a time: p_j = prod_{l != n} a^(l)_{i_l, S} into LDS, then
//    every thread adds p_j p_j^T over its RB x RB block of the padded
//    (16 RB)^2 matrix (rows ty + 16u, columns tx + 16v, so a row of LDS
//    reads is spread over 16 banks) in the accumulation type.  The lower
//    triangle goes to LDS in FP64, lambda_i is added and the system is
//    solved by Cholesky (text after Theorem 1), each thread owning fixed
//    elements of the triangle; one wavefront does the triangular solves.
//  * Rows longer than the plan's threshold are cut into chunks
//    (k_big_chunks, partial records in the accumulation type), summed in
//    chunk order in FP64 by the row's workgroup, so the result does not
//    depend on scheduling.
#include <climits>

#include "dev_common.h"

namespace tfk {

constexpr int BIG_STAGE = 32;   // entries staged per step

// Packed lower triangle of C x C, then C right-hand-side entries.
__host__ __device__ inline int big_record(int C) { return C * (C + 1) / 2 + C; }
__host__ __device__ inline int64_t big_stride(int C) { return ((int64_t)big_record(C) + 3) & ~(int64_t)3; }

// Dynamic LDS of k_big_rows / k_big_chunks: the FP64 system (packed lower
// triangle + right-hand side) or, while entries are accumulated, the staged
// p vectors, their residuals and indices (the two uses do not overlap).
__host__ __device__ inline size_t big_lds(int C, int RB, int ta_bytes, int no)
{
    const size_t sys = (size_t)big_record(C) * 8;
    const size_t stage = (size_t)BIG_STAGE * 16 * RB * ta_bytes + BIG_STAGE * 8 +
                         (size_t)BIG_STAGE * no * 4;
    return sys > stage ? sys : stage;
}

// Gram accumulation of entries [beg, end) of mode n's CSR order: thread
// (ty, tx) ends with acc[u][v] = sum_j p_j[ty + 16u] p_j[tx + 16v] and,
// for tid < C, racc = sum_j rhat_j p_j[tid].
template <int PREC, int RB>
__device__ __forceinline__ void big_accumulate(const BigArgs &a, int64_t beg, int64_t end,
                                               char *smem, const int32_t *cols,
                                               typename Types<PREC>::TA (&acc)[RB][RB],
                                               typename Types<PREC>::TA &racc)
{
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    using TA = typename Types<PREC>::TA;
    constexpr int CPB = 16 * RB;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int C = a.C, K = a.K, no = a.no;
    TA *Ps = reinterpret_cast<TA *>(smem);                                    // [32][CPB]
    double *rs = reinterpret_cast<double *>(smem + (size_t)BIG_STAGE * CPB * sizeof(TA));
    int32_t *is = reinterpret_cast<int32_t *>(rs + BIG_STAGE);               // [32][no]
    const TR *rhat = reinterpret_cast<const TR *>(a.rhat);
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) acc[u][v] = TA(0);
    racc = TA(0);
    for (int64_t q0 = beg; q0 < end; q0 += BIG_STAGE) {
        const int cn = (int)(end - q0 < BIG_STAGE ? end - q0 : BIG_STAGE);
        for (int e = tid; e < cn * no; e += 256) {
            const int ee = e / no, l = e - ee * no;
            int32_t v = 0;
#pragma unroll
            for (int t = 0; t < kMaxModes - 1; ++t)   // static indices into the argument
                if (t == l) v = a.oidx[t][q0 + ee];
            is[e] = v;
        }
        if (tid < cn) {
            const int64_t q = q0 + tid;
            rs[tid] = (double)rhat[a.rperm ? (int64_t)a.rperm[q] : q];
        }
        __syncthreads();
        for (int e = tid; e < cn * CPB; e += 256) {
            const int ee = e / CPB, c = e - ee * CPB;
            TA p = TA(0);
            if (c < C) {
                p = TA(1);
                const int col = cols[c];
#pragma unroll
                for (int l = 0; l < kMaxModes - 1; ++l)
                    if (l < no)
                        p *= (TA)load_f64(reinterpret_cast<const TS *>(a.A[l]) +
                                          (int64_t)is[ee * no + l] * K + col);
            }
            Ps[e] = p;
        }
        __syncthreads();
        for (int j = 0; j < cn; ++j) {
            TA pr[RB], pc[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                pr[u] = Ps[j * CPB + ty + 16 * u];
                pc[u] = Ps[j * CPB + tx + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < RB; ++u)
#pragma unroll
                for (int v = 0; v < RB; ++v) acc[u][v] += pr[u] * pc[v];
            if (tid < C) racc += (TA)rs[j] * Ps[j * CPB + tid];
        }
        __syncthreads();
    }
}

// Partial record of one chunk of a long row (accumulation type).
template <int PREC, int RB>
__global__ __launch_bounds__(256) void k_big_chunks(BigArgs a)
{
    using TA = typename Types<PREC>::TA;
    extern __shared__ __align__(16) char smem[];
    __shared__ int32_t cols[16 * RB];
    if (pass_halted(a.flags)) return;   // uniform: the pass's solves are skipped too
    const Chunk ch = a.chunks[blockIdx.x];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    if (tid < a.C) cols[tid] = a.cols[tid];
    __syncthreads();
    TA acc[RB][RB], racc;
    big_accumulate<PREC, RB>(a, ch.beg, ch.end, smem, cols, acc, racc);
    const int C = a.C;
    TA *out = reinterpret_cast<TA *>(a.gpart) + (int64_t)ch.slot * big_stride(C);
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) {
            const int k1 = ty + 16 * u, k2 = tx + 16 * v;
            if (k1 < C && k2 <= k1) out[k1 * (k1 + 1) / 2 + k2] = acc[u][v];
        }
    if (tid < C) out[C * (C + 1) / 2 + tid] = racc;
}

// One row per workgroup: blocks [0, nsplit) are the chunked rows (their
// records summed in chunk order), then the other non-empty rows, then the
// empty rows (set to zero).
template <int PREC, int RB>
__global__ __launch_bounds__(256) void k_big_rows(BigArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TA = typename Types<PREC>::TA;
    extern __shared__ __align__(16) char smem[];
    __shared__ int32_t cols[16 * RB];
    __shared__ double diag[16 * RB];
    __shared__ int failed;
    constexpr int kOwn = (16 * RB * (16 * RB + 1) / 2 + 255) / 256;
    if (pass_halted(a.flags)) return;   // uniform: no factor changes after a failed pass
    const int C = a.C, K = a.K;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int b = blockIdx.x;
    int row, kind;   // kind 0: entries, 1: chunk records, 2: empty
    if (b < a.nsplit) { row = a.split_rows[b]; kind = 1; }
    else if (b < a.nsplit + a.nitems) { row = a.items[b - a.nsplit]; kind = 0; }
    else { row = a.empty[b - a.nsplit - a.nitems]; kind = 2; }
    if (tid < C) cols[tid] = a.cols[tid];
    if (tid == 0) failed = 0;
    __syncthreads();
    TS *arow = reinterpret_cast<TS *>(a.Aown) + (int64_t)row * K;
    const int64_t beg = a.rowptr[row], end = a.rowptr[row + 1];
    double *L = reinterpret_cast<double *>(smem);    // packed lower triangle
    double *rhs = L + C * (C + 1) / 2;
    const int KT = C * (C + 1) / 2;

    if (kind == 2) {
        // a row with no observed entries is set to zero
        if (tid < C) arow[cols[tid]] = store_cast<TS>(0.0);
    } else {
        if (kind == 0) {
            TA acc[RB][RB], racc;
            big_accumulate<PREC, RB>(a, beg, end, smem, cols, acc, racc);
#pragma unroll
            for (int u = 0; u < RB; ++u)
#pragma unroll
                for (int v = 0; v < RB; ++v) {
                    const int k1 = ty + 16 * u, k2 = tx + 16 * v;
                    if (k1 < C && k2 <= k1) L[k1 * (k1 + 1) / 2 + k2] = (double)acc[u][v];
                }
            if (tid < C) rhs[tid] = (double)racc;
        } else {
            const int64_t gs = big_stride(C);
            const int c0 = a.split_chunk_ptr[b], c1 = a.split_chunk_ptr[b + 1];
            const TA *gp = reinterpret_cast<const TA *>(a.gpart);
            for (int e = tid; e < KT + C; e += 256) {
                double s = 0.0;
                for (int c = c0; c < c1; ++c) s += (double)gp[(int64_t)c * gs + e];
                L[e] = s;   // rhs follows the triangle
            }
        }
        __syncthreads();
        const double lam = a.reg_mode ? a.lambda * (double)(end - beg) : a.lambda;
        for (int k = tid; k < C; k += 256) L[k * (k + 1) / 2 + k] += lam;

        // Cholesky L L^T in place.  Thread tid owns positions tid + 256 t of
        // the packed triangle, decoded once into (row << 8 | column).
        int own[kOwn];
#pragma unroll
        for (int t = 0; t < kOwn; ++t) {
            const int p = tid + 256 * t;
            own[t] = -1;
            if (p < KT) {
                int r = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
                while ((r + 1) * (r + 2) / 2 <= p) ++r;
                while (r * (r + 1) / 2 > p) --r;
                own[t] = (r << 8) | (p - r * (r + 1) / 2);
            }
        }
        for (int j = 0; j < C; ++j) {
            __syncthreads();
            const double d = L[j * (j + 1) / 2 + j];
            const double ljj = sqrt(d > 0.0 ? d : 1.0), rinv = 1.0 / ljj;
            if (tid == 0) {
                diag[j] = ljj;
                if (!(d > 0.0)) failed = 1;
            }
            for (int i = j + 1 + tid; i < C; i += 256) L[i * (i + 1) / 2 + j] *= rinv;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < kOwn; ++t) {
                const int i = own[t] >> 8, k = own[t] & 255;
                if (own[t] >= 0 && k > j)
                    L[i * (i + 1) / 2 + k] -= L[i * (i + 1) / 2 + j] * L[k * (k + 1) / 2 + j];
            }
        }
        __syncthreads();
        if (failed) {
            if (tid == 0) atomicMin(a.bad, (unsigned long long)row);   // the row keeps its value
        } else if (tid < 64) {
            // L y = rhs, then L^T a = y, by one wavefront (its LDS accesses
            // stay in program order, so no barriers)
            for (int k = 0; k < C; ++k) {
                const double yk = rhs[k] / diag[k];
                __builtin_amdgcn_wave_barrier();
                for (int i = k + 1 + tid; i < C; i += 64) rhs[i] -= L[i * (i + 1) / 2 + k] * yk;
                if (tid == 0) rhs[k] = yk;
                __builtin_amdgcn_wave_barrier();
            }
            for (int k = C - 1; k >= 0; --k) {
                const double ak = rhs[k] / diag[k];
                __builtin_amdgcn_wave_barrier();
                for (int i = tid; i < k; i += 64) rhs[i] -= L[k * (k + 1) / 2 + i] * ak;
                if (tid == 0) rhs[k] = ak;
                __builtin_amdgcn_wave_barrier();
            }
            for (int k = tid; k < C; k += 64) arow[cols[k]] = store_cast<TS>(rhs[k]);
        }
    }
}

// R-hat of a split on mode 1's copy (position q in mode 1's CSR order, entry
// j = perm[q]): r += sum_{c in add} prod_n a^(n)_{i_n c} - sum_{c in sub}
// prod_n a^(n)_{i_n c}, in FP64 from the factors (R-hat of Algorithm 1 with
// the pending columns' eq. (SALS_R) folded in).
template <int PREC>
__global__ __launch_bounds__(256) void k_big_boundary(BoundaryArgs a)
{
    using TS = typename Types<PREC>::TS;
    using TR = typename Types<PREC>::TR;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nnz) return;
    const int64_t j = a.perm[q];
    const TS *row[kMaxModes];
#pragma unroll
    for (int n = 0; n < kMaxModes; ++n)   // static indices into the argument
        row[n] = n < a.N ? reinterpret_cast<const TS *>(a.A[n]) + (int64_t)a.idx[j * a.N + n] * a.K
                         : nullptr;
    double add = 0.0, sub = 0.0;
    for (int c = 0; c < a.nadd; ++c) {
        double p = 1.0;
#pragma unroll
        for (int n = 0; n < kMaxModes; ++n)
            if (n < a.N) p *= load_f64(row[n] + a.add[c]);
        add += p;
    }
    for (int c = 0; c < a.nsub; ++c) {
        double p = 1.0;
#pragma unroll
        for (int n = 0; n < kMaxModes; ++n)
            if (n < a.N) p *= load_f64(row[n] + a.sub[c]);
        sub += p;
    }
    TR *r = reinterpret_cast<TR *>(a.r) + q;
    *r = (TR)(((double)*r - sub) + add);
}

template <int PREC, int RB>
static hipError_t big_pass(const BigArgs &a, hipStream_t st)
{
    using TA = typename Types<PREC>::TA;
    const size_t lds = big_lds(a.C, RB, (int)sizeof(TA), a.no);
    if (lds > 65536) {
        // more than 64 KB of dynamic LDS must be allowed per kernel; the
        // attempt's error state is cleared so that it cannot be mistaken for
        // a launch failure below
        hipError_t e = hipFuncSetAttribute((const void *)k_big_rows<PREC, RB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_big_chunks<PREC, RB>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.nchunks > 0) {
        hipLaunchKernelGGL((k_big_chunks<PREC, RB>), dim3(a.nchunks), dim3(256), lds, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (int64_t)a.nsplit + a.nitems + a.nempty;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_big_rows<PREC, RB>), dim3((unsigned)nb), dim3(256), lds, st, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t big_pass_p(const BigArgs &a, hipStream_t st)
{
    if (a.C <= 32) return big_pass<PREC, 2>(a, st);
    if (a.C <= 64) return big_pass<PREC, 4>(a, st);
    if (a.C <= kMaxBigC) return big_pass<PREC, 8>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_big_pass(int prec, const BigArgs &a, hipStream_t st)
{
    if (prec == P_F64) return big_pass_p<P_F64>(a, st);
    if (prec == P_F32) return big_pass_p<P_F32>(a, st);
    return big_pass_p<P_BF16>(a, st);
}

int64_t big_record_stride(int C) { return big_stride(C); }

hipError_t launch_big_boundary(int prec, const BoundaryArgs &a, hipStream_t st)
{
    if (a.nnz == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.nnz + 255) / 256));
    if (prec == P_F64) hipLaunchKernelGGL(k_big_boundary<P_F64>, grid, dim3(256), 0, st, a);
    else if (prec == P_F32) hipLaunchKernelGGL(k_big_boundary<P_F32>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_big_boundary<P_BF16>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace tfk
