// Host-side row planner: turns the CSR offsets of one mode into wavefront
// tasks.  Rows of a mode are independent given the other factors (Section 3.3
// of arXiv:1410.5209); the paper balances them across machines by nonzero
// count (Algorithm 3).  Inside one GPU the same concern becomes: give a row
// as many lanes as its length needs, and cut the longest rows into chunks so
// that no single wavefront holds up the pass.
#include <algorithm>
#include <numeric>

#include "plan.h"
#include "../../include/tf.h"

namespace tfk {

static int lanes_for(int64_t cnt, int lane_nnz)
{
    int64_t need = (cnt + lane_nnz - 1) / lane_nnz;
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    return G;
}

void plan_rows(const int64_t *rowptr, int64_t I, int strategy, int lane_nnz, int split_threshold,
               int chunk_nnz, HostPlan *out)
{
    *out = HostPlan();
    if (lane_nnz <= 0) lane_nnz = 2;
    if (split_threshold <= 0) split_threshold = 4096;
    if (chunk_nnz <= 0) chunk_nnz = 2048;
    auto cnt = [&](int64_t i) { return rowptr[i + 1] - rowptr[i]; };

    if (strategy == TF_STRATEGY_PLAIN) {
        for (int64_t i = 0; i < I; ++i) {
            if (cnt(i) == 0) { out->empty_rows += 1; out->empty.push_back((int32_t)i); continue; }
            out->tasks.push_back(Task{64, (int32_t)out->items.size(), 1, 0});
            out->items.push_back((int32_t)i);
            out->rows_by_lanes[6] += 1;
        }
        out->split_chunk_ptr.push_back(0);
        return;
    }

    std::vector<int32_t> bucket[7];
    std::vector<int32_t> split;
    for (int64_t i = 0; i < I; ++i) {
        const int64_t c = cnt(i);
        if (c == 0) { out->empty_rows += 1; out->empty.push_back((int32_t)i); continue; }
        if (c > split_threshold) { split.push_back((int32_t)i); continue; }
        const int G = lanes_for(c, lane_nnz);
        bucket[__builtin_ctz(G)].push_back((int32_t)i);
    }
    auto heavier = [&](int32_t a, int32_t b) { return cnt(a) > cnt(b); };

    // long rows first, cut into chunks of chunk_nnz entries (larger for the
    // longest rows, so that no row has more than kMaxChunksPerRow chunks and
    // the fixed-order sum of its partials stays short)
    std::stable_sort(split.begin(), split.end(), heavier);
    for (int32_t row : split) {
        out->split_rows.push_back(row);
        out->split_chunk_ptr.push_back((int32_t)out->chunks.size());
        const int64_t len = std::max<int64_t>(chunk_nnz, (cnt(row) + kMaxChunksPerRow - 1) / kMaxChunksPerRow);
        for (int64_t b = rowptr[row]; b < rowptr[row + 1]; b += len) {
            const int64_t e = std::min<int64_t>(b + len, rowptr[row + 1]);
            const int32_t slot = (int32_t)out->chunks.size();
            out->tasks.push_back(Task{64, slot, 1, 1});
            out->chunks.push_back(Chunk{row, (int32_t)b, (int32_t)e, slot});
        }
    }
    out->split_chunk_ptr.push_back((int32_t)out->chunks.size());

    // then rows by lanes per row, widest first; rows of similar length share
    // a wavefront so that its groups finish together
    for (int b = 6; b >= 0; --b) {
        const int G = 1 << b;
        const int per = 64 / G;
        std::stable_sort(bucket[b].begin(), bucket[b].end(), heavier);
        out->rows_by_lanes[b] = (int64_t)bucket[b].size();
        for (size_t s = 0; s < bucket[b].size(); s += per) {
            const int count = (int)std::min<size_t>(per, bucket[b].size() - s);
            out->tasks.push_back(Task{G, (int32_t)out->items.size(), count, 0});
            for (int q = 0; q < count; ++q) out->items.push_back(bucket[b][s + q]);
        }
    }
}

int pick_cp(int C, int prec)
{
    static const int f64[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    static const int f32[] = {1, 2, 4, 5, 8, 10, 12, 16, 32};
    if (prec == 0) {
        for (int v : f64) if (v >= C) return v;
    } else {
        for (int v : f32) if (v >= C) return v;
    }
    return -1;
}

}  // namespace tfk

extern "C" tf_status tf_plan_rows(const int64_t *rowptr, int64_t I, int32_t strategy,
                                  int32_t lane_nnz, int32_t split_threshold, int32_t chunk_nnz,
                                  tf_plan_summary *out)
{
    if (!rowptr || !out || I < 1 || (strategy != TF_STRATEGY_PLAIN && strategy != TF_STRATEGY_SKEW))
        return TF_E_INVALID;
    for (int64_t i = 0; i < I; ++i)
        if (rowptr[i + 1] < rowptr[i]) return TF_E_INVALID;
    if (rowptr[0] != 0) return TF_E_INVALID;
    tfk::HostPlan p;
    tfk::plan_rows(rowptr, I, strategy, lane_nnz, split_threshold, chunk_nnz, &p);
    out->tasks = (int64_t)p.tasks.size();
    out->split_rows = (int64_t)p.split_rows.size();
    out->chunks = (int64_t)p.chunks.size();
    out->empty_rows = p.empty_rows;
    for (int b = 0; b < 7; ++b) out->rows_by_lanes[b] = p.rows_by_lanes[b];
    return TF_OK;
}
