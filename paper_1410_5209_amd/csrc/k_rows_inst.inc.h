// Instantiates the row kernels of one precision (TF_PREC_ID) for its compute
// widths (TF_CP_LIST) and every number of other modes (1..7).
#pragma once

#include "k_rows.inc.h"
#include "k_rows_wide.inc.h"

#include <algorithm>

namespace tfk {

// Launch of a row-accumulation kernel: a grid of one wavefront per task, or
// (persistent launch, a.work set) as many workgroups as the GPU holds at
// once, whose wavefronts take tasks from the work counter.
template <typename F>
static hipError_t launch_rows(F *kernel, const AccumArgs &a, int grid, hipStream_t st)
{
    if (a.work) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        grid = std::max(1, std::min(grid, per_cu * cus));
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int PREC, int CP, int NO>
static hipError_t accum_no(bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    bool any_before = false;
    for (int l = 0; l < NO; ++l) any_before |= a.before[l] != 0;
    if (first && any_before) return launch_rows(k_accum<PREC, CP, NO, 2>, a, grid, st);
    if (first) return launch_rows(k_accum<PREC, CP, NO, 1>, a, grid, st);
    return launch_rows(k_accum<PREC, CP, NO, 0>, a, grid, st);
}

template <int PREC, int CP>
static hipError_t accum_cp(int no, bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    switch (no) {
    case 1: return accum_no<PREC, CP, 1>(first, a, grid, st);
    case 2: return accum_no<PREC, CP, 2>(first, a, grid, st);
    case 3: return accum_no<PREC, CP, 3>(first, a, grid, st);
    case 4: return accum_no<PREC, CP, 4>(first, a, grid, st);
    case 5: return accum_no<PREC, CP, 5>(first, a, grid, st);
    case 6: return accum_no<PREC, CP, 6>(first, a, grid, st);
    case 7: return accum_no<PREC, CP, 7>(first, a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC, int CP>
static hipError_t solve_cp(const SolveArgs &a, hipStream_t st)
{
    const int grid = (int)((a.I + 255) / 256);
    hipLaunchKernelGGL((k_solve<PREC, CP>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int PREC, int CP>
static hipError_t reduce_cp(const int32_t *rows, const int32_t *ptr, int nsplit, const void *gpart,
                            void *gram, hipStream_t st)
{
    hipLaunchKernelGGL((k_chunk_reduce<PREC, CP>), dim3(nsplit), dim3(256), 0, st, rows, ptr,
                       gpart, gram);
    return hipGetLastError();
}

template <int PREC, int NO>
static hipError_t accum_wide_no(bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    bool any_before = false;
    for (int l = 0; l < NO; ++l) any_before |= a.before[l] != 0;
    if (first && any_before) return launch_rows(k_accum_wide<PREC, NO, 2>, a, grid, st);
    if (first) return launch_rows(k_accum_wide<PREC, NO, 1>, a, grid, st);
    return launch_rows(k_accum_wide<PREC, NO, 0>, a, grid, st);
}

template <int PREC, int CP>
static hipError_t accum_wide(int no, bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    switch (no) {
    case 1: return accum_wide_no<PREC, 1>(first, a, grid, st);
    case 2: return accum_wide_no<PREC, 2>(first, a, grid, st);
    case 3: return accum_wide_no<PREC, 3>(first, a, grid, st);
    case 4: return accum_wide_no<PREC, 4>(first, a, grid, st);
    case 5: return accum_wide_no<PREC, 5>(first, a, grid, st);
    case 6: return accum_wide_no<PREC, 6>(first, a, grid, st);
    case 7: return accum_wide_no<PREC, 7>(first, a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC, int CP>
static hipError_t solve_wide(const SolveArgs &a, hipStream_t st)
{
    const int grid = (int)((a.I + 7) / 8);
    hipLaunchKernelGGL((k_solve_wide<PREC>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace tfk

#define TF_CP_CASE(FN, CPV, ...) \
    case CPV: return FN<TF_PREC_ID, CPV>(__VA_ARGS__);
