// Row kernels, precision f32.
#define TF_PREC_ID tfk::P_F32
#include "k_rows_inst.inc.h"

namespace tfk {

hipError_t launch_accum_f32(int CP, int no, bool first, const AccumArgs &a, int grid, hipStream_t st)
{
    switch (CP) {
    TF_CP_CASE(accum_cp, 1, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 2, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 4, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 5, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 8, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 10, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 12, no, first, a, grid, st)
    TF_CP_CASE(accum_cp, 16, no, first, a, grid, st)
    TF_CP_CASE(accum_wide, 32, no, first, a, grid, st)
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_f32(int CP, const SolveArgs &a, hipStream_t st)
{
    switch (CP) {
    TF_CP_CASE(solve_cp, 1, a, st)
    TF_CP_CASE(solve_cp, 2, a, st)
    TF_CP_CASE(solve_cp, 4, a, st)
    TF_CP_CASE(solve_cp, 5, a, st)
    TF_CP_CASE(solve_cp, 8, a, st)
    TF_CP_CASE(solve_cp, 10, a, st)
    TF_CP_CASE(solve_cp, 12, a, st)
    TF_CP_CASE(solve_cp, 16, a, st)
    TF_CP_CASE(solve_wide, 32, a, st)
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_f32(int CP, const int32_t *rows, const int32_t *ptr, int nsplit, const void *gpart, void *gram, hipStream_t st)
{
    switch (CP) {
    TF_CP_CASE(reduce_cp, 1, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 2, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 4, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 5, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 8, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 10, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 12, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 16, rows, ptr, nsplit, gpart, gram, st)
    TF_CP_CASE(reduce_cp, 32, rows, ptr, nsplit, gpart, gram, st)
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tfk
