// Host-side row planner of a mode pass (no HIP types: it also builds with a
// plain C++ compiler, e.g. for sanitizer runs on the CPU).
#pragma once

#include <cstdint>
#include <vector>

namespace tfk {

// A task is one wavefront's unit of work.
//   kind 0: up to 64/G rows, G lanes each (items[base .. base+count))
//   kind 1: one chunk of a long row (chunks[base]), 64 lanes
struct Task {
    int32_t G;
    int32_t base;
    int32_t count;
    int32_t kind;
};
struct Chunk {
    int32_t row;
    int32_t beg;
    int32_t end;
    int32_t slot;
};

constexpr int64_t kMaxChunksPerRow = 1024;

struct HostPlan {
    std::vector<Task> tasks;
    std::vector<int32_t> items;
    std::vector<Chunk> chunks;
    std::vector<int32_t> split_rows;     // rows cut into chunks
    std::vector<int32_t> split_chunk_ptr;// chunk range per split row (size+1)
    std::vector<int32_t> empty;          // rows with no entries
    int64_t empty_rows = 0;
    int64_t rows_by_lanes[7] = {0, 0, 0, 0, 0, 0, 0};
};

void plan_rows(const int64_t *rowptr, int64_t I, int strategy, int lane_nnz, int split_threshold,
               int chunk_nnz, HostPlan *out);

// Compute widths the row kernels are instantiated for; C is padded up to the
// next one (padded slab columns hold zeros, which leaves the solution of the
// real columns unchanged and the padded ones at zero).  -1: no register or
// wide kernel takes C (the workgroup-per-row kernels do, up to kMaxBigC).
int pick_cp(int C, int prec);

}  // namespace tfk
