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
    int32_t *req_status;          // NULL, or out nreq: TF_OK / TF_E_NUMERIC per request
    // full rank: the entries of request q are cut into chunks of
    // kFoldChunkEntries; chunk_first[q] .. chunk_first[q + 1] - 1 are its
    // chunks, chunk_req[c] the request of chunk c; gpart holds one partial
    // Gram record per chunk (kFoldGramStride(K) accumulation-type values)
    const int32_t *chunk_first;   // nreq + 1
    const int32_t *chunk_req;     // nchunks
    int32_t nchunks;
    void *gpart;
};

constexpr int kFoldChunkEntries = 256;
constexpr int kFoldMaxKFull = 128;
// Both methods start from the request's Gram matrix when K <= 128 (chunk
// records); CDTF above that walks the entries (needs the r workspace).
inline bool fold_uses_gram(int K) { return K <= kFoldMaxKFull; }
// Partial Gram record: lower triangle of B (K (K + 1) / 2) then c (K).
__host__ __device__ inline int64_t fold_gram_stride(int K) { return ((int64_t)K * (K + 1) / 2 + K + 3) & ~(int64_t)3; }
// Chunks of a batch: sum over requests of ceil(m_q / kFoldChunkEntries).
inline int64_t fold_chunks(const int64_t *h_req_ptr, int64_t nreq)
{
    int64_t n = 0;
    for (int64_t q = 0; q < nreq; ++q)
        n += (h_req_ptr[q + 1] - h_req_ptr[q] + kFoldChunkEntries - 1) / kFoldChunkEntries;
    return n;
}
// Fill chunk_first (nreq + 1) and chunk_req (fold_chunks entries) on the host.
inline void fold_chunk_tables(const int64_t *h_req_ptr, int64_t nreq, int32_t *first, int32_t *req)
{
    int32_t c = 0;
    for (int64_t q = 0; q < nreq; ++q) {
        first[q] = c;
        const int64_t n = (h_req_ptr[q + 1] - h_req_ptr[q] + kFoldChunkEntries - 1) / kFoldChunkEntries;
        for (int64_t t = 0; t < n; ++t) req[c++] = (int32_t)q;
    }
    first[nreq] = c;
}

size_t fold_full_lds(int K, int prec);
// Device address of the fold-in scratch array on `device` (looked up once,
// with that device current); its size in bytes.
hipError_t fold_scratch_setup(int device);
size_t fold_scratch_bytes();
// Validation must complete (and pass) before compute: the compute kernels
// index the factors with the request's indices.
hipError_t launch_fold_validate(const FoldArgs &a, int64_t total, const int64_t *dims,
                                hipStream_t st);
hipError_t launch_fold_compute(int prec, const FoldArgs &a, int64_t total, int method,
                               hipStream_t st);

}  // namespace tfk
