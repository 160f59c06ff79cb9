// Host sanitizer run of the row planner: random row-length profiles (empty
// rows, uniform, Zipf-like heavy tails, one row beyond the chunk cap) through
// both strategies and a range of tiles, checking that the plan covers every
// non-empty row exactly once and that every chunk stays inside its row.
// Built with -fsanitize=address,undefined by the CPU tests.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1410_5209_amd/csrc/plan.h"
#include "../../include/tf.h"

#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            std::exit(1);                                                      \
        }                                                                      \
    } while (0)

static void check_plan(const std::vector<int64_t> &rp, int strategy, int lane, int thr, int chunk)
{
    const int64_t I = (int64_t)rp.size() - 1;
    tfk::HostPlan p;
    tfk::plan_rows(rp.data(), I, strategy, lane, thr, chunk, &p);
    std::vector<int> seen(I, 0);
    for (const auto &t : p.tasks) {
        CHECK(t.G >= 1 && t.G <= 64 && (t.G & (t.G - 1)) == 0);
        if (t.kind == 0) {
            CHECK(t.count >= 1 && t.count <= 64 / t.G);
            CHECK(t.base >= 0 && (size_t)(t.base + t.count) <= p.items.size());
        } else {
            CHECK(t.kind == 1 && t.count == 1 && t.base >= 0 && (size_t)t.base < p.chunks.size());
        }
    }
    for (int32_t r : p.items) { CHECK(r >= 0 && r < I); seen[r] += 1; }
    CHECK(p.split_chunk_ptr.size() == p.split_rows.size() + 1);
    for (size_t s = 0; s < p.split_rows.size(); ++s) {
        const int32_t r = p.split_rows[s];
        CHECK(r >= 0 && r < I);
        seen[r] += 1;
        int64_t at = rp[r];
        const int32_t c0 = p.split_chunk_ptr[s], c1 = p.split_chunk_ptr[s + 1];
        CHECK(c1 > c0 && c1 - c0 <= tfk::kMaxChunksPerRow);
        for (int32_t c = c0; c < c1; ++c) {
            const tfk::Chunk &ch = p.chunks[c];
            CHECK(ch.row == r && ch.slot == c && ch.beg == at && ch.end > ch.beg);
            at = ch.end;
        }
        CHECK(at == rp[r + 1]);
    }
    int64_t empty = 0;
    for (int32_t r : p.empty) { CHECK(rp[r + 1] == rp[r]); seen[r] += 1; ++empty; }
    CHECK(empty == p.empty_rows);
    for (int64_t i = 0; i < I; ++i) CHECK(seen[i] == 1);
    tf_plan_summary sum;
    CHECK(tf_plan_rows(rp.data(), I, strategy, lane, thr, chunk, &sum) == TF_OK);
    CHECK(sum.tasks == (int64_t)p.tasks.size() && sum.chunks == (int64_t)p.chunks.size());
}

int main()
{
    std::mt19937_64 g(7);
    for (int trial = 0; trial < 60; ++trial) {
        const int64_t I = 1 + (int64_t)(g() % 3000);
        std::vector<int64_t> rp(I + 1, 0);
        for (int64_t i = 0; i < I; ++i) {
            int64_t len;
            switch (trial % 4) {
            case 0: len = (int64_t)(g() % 5); break;                         // many empty rows
            case 1: len = 50 + (int64_t)(g() % 100); break;                  // uniform
            case 2: len = (int64_t)(20000.0 / (double)(1 + (g() % I))); break;  // heavy tail
            default: len = i == 0 ? 3000000 : (int64_t)(g() % 8); break;    // one row past the chunk cap
            }
            rp[i + 1] = rp[i] + len;
        }
        const int lanes[] = {1, 2, 4, 8};
        const int chunks[] = {64, 1024, 4096};
        check_plan(rp, TF_STRATEGY_PLAIN, 2, 4096, 2048);
        check_plan(rp, TF_STRATEGY_SKEW, lanes[trial % 4], 2 * chunks[trial % 3], chunks[trial % 3]);
        check_plan(rp, TF_STRATEGY_SKEW, 0, 0, 0);
    }
    std::vector<int64_t> bad = {0, 3, 2};
    tf_plan_summary s;
    CHECK(tf_plan_rows(bad.data(), 2, TF_STRATEGY_SKEW, 2, 4096, 2048, &s) == TF_E_INVALID);
    std::printf("sanitized planner ok\n");
    return 0;
}
