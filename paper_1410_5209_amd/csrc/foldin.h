// Fold-in kernels and the serving loop built on them (internal).
#pragma once

#include "tf_internal.h"

namespace tfk {

struct Dims8x { int64_t d[kMaxModes]; };

struct FoldArgs {
    int32_t N, mode, K, nreq;
    const int64_t *req_ptr;       // device, nreq + 1 entry offsets
    const int32_t *oidx;          // device, total x (N - 1), other modes ascending
    const double *vals;           // device, total
    const void *A[kMaxModes];     // resident factors (storage type)
    void *P;                      // workspace, total x K (accumulation type)
    double *r;                    // workspace, total (CDTF only)
    double *rows;                 // out, nreq x K
    double lambda;
    int32_t reg_mode;
    int32_t sweeps;
    unsigned long long *bad;      // first bad entry (validation)
    unsigned long long *bad_req;  // first request whose Cholesky failed
};

size_t fold_full_lds(int K, int prec);
// Validation must complete (and pass) before compute: the compute kernels
// index the factors with the request's indices.
hipError_t launch_fold_validate(const FoldArgs &a, int64_t total, const int64_t *dims,
                                hipStream_t st);
hipError_t launch_fold_compute(int prec, const FoldArgs &a, int64_t total, int method,
                               hipStream_t st);

constexpr int kFoldMaxKFull = 128;

}  // namespace tfk
