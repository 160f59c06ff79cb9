// Fold-in entry points: the synchronous batched call and the serving loop.
//
// Serving: submit() copies a request into the queue.  A scheduler thread
// waits until a stream slot is free, then takes queued requests in arrival
// order while their device bytes fit the slot's arena (admission by memory)
// and the batch is below max_batch, stages them in pinned host memory,
// copies them to the slot's arena, launches the fold-in kernels and the
// copy-back on the slot's stream, and records an event.  One completion
// thread per slot waits for that event, stamps the requests, hands the rows
// to their waiters and frees the slot.  With two or more slots, batches that
// arrive while others run are admitted as slots and memory free up, and their
// work overlaps on the device (continuous batching).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
#include <vector>

#include "foldin.h"

using namespace tfk;
using clk = std::chrono::steady_clock;

namespace {

size_t ta_bytes(int prec) { return prec == P_F64 ? 8 : 4; }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Upper bound on the chunks of a batch (each request: ceil(m / chunk)).
int64_t max_chunks(int64_t nreq, int64_t total) { return nreq + total / kFoldChunkEntries; }

// Device bytes a batch needs (arena layout below; the first five parts are
// staged in the same layout in pinned memory and copied in one transfer).
size_t batch_bytes(int N, int K, int prec, int method, int64_t nreq, int64_t total)
{
    (void)method;
    const int64_t nc = fold_uses_gram(K) ? max_chunks(nreq, total) : 0;
    size_t b = align256((size_t)(nreq + 1) * 8);                  // req_ptr
    b += align256((size_t)(nreq + 1) * 4);                        // chunk_first
    b += align256((size_t)nc * 4);                                // chunk_req
    b += align256((size_t)total * (N - 1) * 4);                   // indices
    b += align256((size_t)total * 8);                             // values
    b += align256((size_t)total * K * ta_bytes(prec));            // P
    if (!fold_uses_gram(K)) b += align256((size_t)total * 8);     // r (CDTF, large K)
    b += align256((size_t)nc * fold_gram_stride(K) * ta_bytes(prec));  // partial Grams
    b += align256((size_t)nreq * K * 8);                          // rows
    b += align256((size_t)nreq * 4);                              // per-request status
    b += 256;                                                     // flags
    return b;
}

struct Arena {
    int64_t *req_ptr;
    int32_t *chunk_first;
    int32_t *chunk_req;
    int32_t *oidx;
    double *vals;
    void *P;
    double *r;
    void *gpart;
    double *rows;
    int32_t *status;
    unsigned long long *flags;
};

Arena carve(void *base, int N, int K, int prec, int method, int64_t nreq, int64_t total)
{
    (void)method;
    const int64_t nc = fold_uses_gram(K) ? max_chunks(nreq, total) : 0;
    char *p = static_cast<char *>(base);
    Arena a{};
    a.req_ptr = reinterpret_cast<int64_t *>(p); p += align256((size_t)(nreq + 1) * 8);
    a.chunk_first = reinterpret_cast<int32_t *>(p); p += align256((size_t)(nreq + 1) * 4);
    a.chunk_req = reinterpret_cast<int32_t *>(p); p += align256((size_t)nc * 4);
    a.oidx = reinterpret_cast<int32_t *>(p); p += align256((size_t)total * (N - 1) * 4);
    a.vals = reinterpret_cast<double *>(p); p += align256((size_t)total * 8);
    a.P = p; p += align256((size_t)total * K * ta_bytes(prec));
    a.r = nullptr;
    if (!fold_uses_gram(K)) { a.r = reinterpret_cast<double *>(p); p += align256((size_t)total * 8); }
    a.gpart = p; p += align256((size_t)nc * fold_gram_stride(K) * ta_bytes(prec));
    a.rows = reinterpret_cast<double *>(p); p += align256((size_t)nreq * K * 8);
    a.status = reinterpret_cast<int32_t *>(p); p += align256((size_t)nreq * 4);
    a.flags = reinterpret_cast<unsigned long long *>(p);
    return a;
}

FoldArgs fold_args(const tf_ctx *c, int mode, const Arena &ar, int64_t nreq, int sweeps)
{
    FoldArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = c->N;
    a.mode = mode;
    a.K = c->K;
    a.nreq = (int32_t)nreq;
    a.req_ptr = ar.req_ptr;
    a.oidx = ar.oidx;
    a.vals = ar.vals;
    for (int n = 0; n < c->N; ++n) a.A[n] = c->m[n].A;
    a.P = ar.P;
    a.r = ar.r;
    a.rows = ar.rows;
    a.lambda = c->lambda;
    a.reg_mode = c->opt.reg_mode;
    a.sweeps = sweeps;
    a.bad = ar.flags;
    a.bad_req = ar.flags + 1;
    a.req_status = ar.status;
    a.chunk_first = ar.chunk_first;
    a.chunk_req = ar.chunk_req;
    a.gpart = ar.gpart;
    return a;
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

// ------------------------------------------------------------------ server
struct SReq {
    int64_t m = 0;
    std::vector<int32_t> idx;
    std::vector<double> vals;
    std::vector<double> row;
    clk::time_point t_submit, t_launch, t_done;
    int batch_size = 0;
    int status = TF_OK;
    bool done = false;
};

struct SSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    void *dev = nullptr;
    char *hin = nullptr;       // pinned staging of inputs
    char *hout = nullptr;      // pinned rows, then per-request status words
    std::vector<SReq *> batch;
    bool busy = false;         // owned by a batch (set by scheduler)
    bool launched = false;     // work enqueued, completer may wait
    bool failed = false;       // a HIP call of the batch failed: no row is valid
    std::string fail_msg;
    std::thread completer;
};

struct tf_server {
    tf_ctx *ctx = nullptr;
    tf_serve_opts o{};
    size_t slot_bytes = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_slot;
    std::deque<SReq *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<SReq>> reqs;
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<SSlot>> slots;
    bool closing = false, stop = false;
    std::thread sched;
    // statistics
    std::vector<double> lat_us;
    bool have_first = false;
    clk::time_point t_first, t_last;
    int64_t batches = 0, busy_rejects = 0, max_queue = 0;
    double batch_sum = 0.0;
    int64_t failed = 0;        // requests completed with TF_E_DEVICE
    std::atomic<int32_t> inject{0};  // batches left to fail on purpose (tf_serve_inject_fault)
    std::string err;
};

namespace {

size_t req_bytes(const tf_server *s, int64_t m)
{
    const tf_ctx *c = s->ctx;
    const size_t chunks = fold_uses_gram(c->K) ? (size_t)max_chunks(1, m) : 0;
    return (size_t)m * ((c->N - 1) * 4 + 8 + (size_t)c->K * ta_bytes(c->prec) +
                        (fold_uses_gram(c->K) ? 0 : 8)) + (size_t)c->K * 8 + 8 + 1024 +
           chunks * (4 + (size_t)fold_gram_stride(c->K) * ta_bytes(c->prec));
}

// Stage and enqueue one batch on the slot's stream.  Every HIP call is
// checked; on a failure the batch is marked failed (its requests complete
// with TF_E_DEVICE and no row is read back) and the message is kept.
void run_batch(tf_server *s, SSlot &slot)
{
    tf_ctx *c = s->ctx;
    const int N = c->N, K = c->K;
    const int64_t nreq = (int64_t)slot.batch.size();
    int64_t total = 0;
    for (SReq *r : slot.batch) total += r->m;
    // stage inputs in pinned memory in the arena's layout:
    // req_ptr | chunk_first | chunk_req | indices | values
    Arena hs = carve(slot.hin, N, K, c->prec, s->o.method, nreq, total);
    int64_t *hp = hs.req_ptr;
    int32_t *hi = hs.oidx;
    double *hv = hs.vals;
    hp[0] = 0;
    int64_t off = 0;
    for (int64_t q = 0; q < nreq; ++q) {
        SReq *r = slot.batch[q];
        if (r->m) {
            std::memcpy(hi + off * (N - 1), r->idx.data(), (size_t)r->m * (N - 1) * 4);
            std::memcpy(hv + off, r->vals.data(), (size_t)r->m * 8);
        }
        off += r->m;
        hp[q + 1] = off;
    }
    int64_t nchunks = 0;
    if (fold_uses_gram(K)) {
        nchunks = fold_chunks(hp, nreq);
        fold_chunk_tables(hp, nreq, hs.chunk_first, hs.chunk_req);
    }
    Arena ar = carve(slot.dev, N, K, c->prec, s->o.method, nreq, total);
    const size_t in_bytes = (size_t)((char *)(hv + total) - slot.hin);
    const size_t out_bytes = (size_t)((char *)(ar.status + nreq) - (char *)ar.rows);
    slot.failed = false;
    slot.fail_msg.clear();
    const char *step = "input copy";
    hipError_t e = hipMemcpyAsync(ar.req_ptr, slot.hin, in_bytes, hipMemcpyHostToDevice, slot.st);
    if (e == hipSuccess) {
        FoldArgs a = fold_args(c, s->o.mode, ar, nreq, s->o.sweeps);
        a.nchunks = (int32_t)nchunks;
        step = "fold-in launch";
        int32_t left = s->inject.load();
        while (left > 0 && !s->inject.compare_exchange_weak(left, left - 1)) {}
        e = left > 0 ? hipErrorLaunchFailure : launch_fold_compute(c->prec, a, total, s->o.method, slot.st);
    }
    if (e == hipSuccess) {
        step = "row copy-back";
        e = hipMemcpyAsync(slot.hout, ar.rows, out_bytes, hipMemcpyDeviceToHost, slot.st);
    }
    if (e == hipSuccess) {
        step = "event record";
        e = hipEventRecord(slot.ev, slot.st);
    }
    if (e != hipSuccess) {
        slot.failed = true;
        slot.fail_msg = std::string("serving batch: ") + step + " failed: " + hipGetErrorString(e);
    }
}

void scheduler(tf_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        SSlot *free_slot = nullptr;
        s->cv_sched.wait(lk, [&] {
            if (s->stop) return true;
            if (s->queue.empty()) return false;
            for (auto &sl : s->slots)
                if (!sl->busy) { free_slot = sl.get(); return true; }
            return false;
        });
        if (s->stop) break;
        // admission: arrival order, by memory and batch size
        int64_t nreq = 0, total = 0;
        std::vector<SReq *> batch;
        while (!s->queue.empty() && (int)batch.size() < s->o.max_batch) {
            SReq *r = s->queue.front();
            const size_t need = batch_bytes(s->ctx->N, s->ctx->K, s->ctx->prec, s->o.method,
                                            nreq + 1, total + r->m);
            if (!batch.empty() && need > s->slot_bytes) break;
            batch.push_back(r);
            s->queue.pop_front();
            nreq += 1;
            total += r->m;
        }
        free_slot->busy = true;
        free_slot->batch = std::move(batch);
        const clk::time_point now = clk::now();
        for (SReq *r : free_slot->batch) {
            r->t_launch = now;
            r->batch_size = (int)nreq;
        }
        s->batches += 1;
        s->batch_sum += (double)nreq;
        lk.unlock();
        run_batch(s, *free_slot);
        lk.lock();
        free_slot->launched = true;
        s->cv_slot.notify_all();
    }
}

void completer(tf_server *s, SSlot *slot)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_slot.wait(lk, [&] { return s->stop || slot->launched; });
        if (!slot->launched) break;   // stop with nothing in flight
        lk.unlock();
        // a failed batch: drain what was enqueued before the failure, so the
        // slot's buffers are idle before the next batch, and read nothing back
        const bool failed = slot->failed;
        if (failed) (void)hipStreamSynchronize(slot->st);
        else (void)hipEventSynchronize(slot->ev);
        const clk::time_point now = clk::now();
        const int K = s->ctx->K;
        const size_t nreq = slot->batch.size();
        const double *rows = reinterpret_cast<const double *>(slot->hout);
        const int32_t *status = reinterpret_cast<const int32_t *>(slot->hout + align256(nreq * (size_t)K * 8));
        lk.lock();
        if (failed) s->err = slot->fail_msg;
        for (size_t q = 0; q < nreq; ++q) {
            SReq *r = slot->batch[q];
            if (failed) {
                r->row.assign((size_t)K, std::nan(""));
                r->status = TF_E_DEVICE;
                s->failed += 1;
            } else {
                r->row.assign(rows + q * K, rows + (q + 1) * K);
                r->status = status[q] == TF_OK ? TF_OK : TF_E_NUMERIC;
            }
            r->t_done = now;
            r->done = true;
            s->lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        }
        s->t_last = now;
        slot->batch.clear();
        slot->launched = false;
        slot->busy = false;
        s->cv_done.notify_all();
        s->cv_sched.notify_all();
    }
}

void destroy_server(tf_server *s)
{
    for (auto &sl : s->slots) {
        if (sl->ev) (void)hipEventDestroy(sl->ev);
        if (sl->st) (void)hipStreamDestroy(sl->st);
        if (sl->dev) ctx_free(s->ctx, sl->dev);
        if (sl->hin) (void)hipHostFree(sl->hin);
        if (sl->hout) (void)hipHostFree(sl->hout);
    }
    delete s;
}

}  // namespace

extern "C" {

void tf_serve_default_options(tf_serve_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->size = sizeof(tf_serve_opts);
    o->mode = 0;
    o->method = TF_FOLDIN_FULL;
    o->sweeps = 3;
    o->streams = 2;
    o->max_batch = 512;
    o->queue_cap = 65536;
    o->mem_budget = (int64_t)1 << 30;
}

tf_status tf_serve_open(tf_ctx *ctx, const tf_serve_opts *opts, tf_server **out)
{
    if (!ctx || !out) return TF_E_INVALID;
    *out = nullptr;
    tf_serve_opts o;
    tf_serve_default_options(&o);
    if (opts) {
        if (opts->size != sizeof(tf_serve_opts)) {
            ctx->err = "tf_serve_opts.size mismatch";
            return TF_E_INVALID;
        }
        o = *opts;
    }
    if (o.mode < 0 || o.mode >= ctx->N || (o.method != TF_FOLDIN_FULL && o.method != TF_FOLDIN_CDTF) ||
        o.streams < 1 || o.streams > 16 || o.max_batch < 1 || o.queue_cap < 1 || o.mem_budget <= 0 ||
        (o.method == TF_FOLDIN_CDTF && o.sweeps < 1)) {
        ctx->err = "bad serving options";
        return TF_E_INVALID;
    }
    if (o.method == TF_FOLDIN_FULL && ctx->K > kFoldMaxKFull) {
        ctx->err = "full-rank fold-in supports K <= 128";
        return TF_E_UNSUPPORTED;
    }
    tf_server *s = new tf_server();
    s->ctx = ctx;
    s->o = o;
    s->slot_bytes = (size_t)(o.mem_budget / o.streams);
    for (int i = 0; i < o.streams; ++i) {
        auto sl = std::make_unique<SSlot>();
        hipError_t e = hipStreamCreate(&sl->st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming);
        if (e == hipSuccess) e = ctx_alloc(ctx, &sl->dev, s->slot_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl->hin, s->slot_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl->hout,
                              align256((size_t)o.max_batch * ctx->K * 8) + (size_t)o.max_batch * 4,
                              hipHostMallocDefault);
        s->slots.push_back(std::move(sl));
        if (e != hipSuccess) {
            ctx->err = std::string("serving resources: ") + hipGetErrorString(e);
            destroy_server(s);
            return e == hipErrorOutOfMemory ? TF_E_NOMEM : TF_E_DEVICE;
        }
    }
    s->sched = std::thread(scheduler, s);
    for (auto &sl : s->slots) sl->completer = std::thread(completer, s, sl.get());
    *out = s;
    return TF_OK;
}

tf_status tf_serve_submit(tf_server *s, const tf_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket || req->m < 0 || (req->m > 0 && (!req->h_idx || !req->h_vals)))
        return TF_E_INVALID;
    const tf_ctx *c = s->ctx;
    const int N = c->N;
    // host-side validation (the kernels index the factors with these)
    for (int64_t j = 0; j < req->m; ++j) {
        if (!std::isfinite(req->h_vals[j])) return TF_E_INVALID;
        int q = 0;
        for (int l = 0; l < N; ++l) {
            if (l == s->o.mode) continue;
            const int32_t v = req->h_idx[j * (N - 1) + q];
            if (v < 0 || (int64_t)v >= c->dims[l]) return TF_E_INVALID;
            ++q;
        }
    }
    if (batch_bytes(N, c->K, c->prec, s->o.method, 1, req->m) > s->slot_bytes ||
        req_bytes(s, req->m) > s->slot_bytes)
        return TF_E_INVALID;
    auto r = std::make_unique<SReq>();
    r->m = req->m;
    r->idx.assign(req->h_idx, req->h_idx + (size_t)req->m * (N - 1));
    r->vals.assign(req->h_vals, req->h_vals + req->m);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) return TF_E_STATE;
    if ((int64_t)s->queue.size() >= s->o.queue_cap) {
        s->busy_rejects += 1;
        return TF_E_BUSY;
    }
    r->t_submit = clk::now();
    if (!s->have_first) { s->t_first = r->t_submit; s->have_first = true; }
    const uint64_t t = s->next_ticket++;
    s->queue.push_back(r.get());
    s->reqs.emplace(t, std::move(r));
    s->max_queue = std::max<int64_t>(s->max_queue, (int64_t)s->queue.size());
    *ticket = t;
    s->cv_sched.notify_one();
    return TF_OK;
}

tf_status tf_serve_wait(tf_server *s, uint64_t ticket, double *h_row, tf_req_stats *st)
{
    if (!s) return TF_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return TF_E_INVALID;
    SReq *r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->done; });
    if (h_row) std::memcpy(h_row, r->row.data(), (size_t)s->ctx->K * 8);
    if (st) {
        st->latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
        st->queue_us = std::chrono::duration<double, std::micro>(r->t_launch - r->t_submit).count();
        st->batch_size = r->batch_size;
        st->status = r->status;
    }
    const tf_status rs = r->status;
    s->reqs.erase(it);
    return rs;
}

tf_status tf_serve_replay(tf_server *s, int64_t nreq, const double *h_arrival_s,
                          const tf_request *reqs, uint64_t *tickets)
{
    if (!s || nreq < 0 || (nreq > 0 && (!h_arrival_s || !reqs || !tickets))) return TF_E_INVALID;
    const clk::time_point t0 = clk::now();
    for (int64_t i = 0; i < nreq; ++i) {
        const clk::time_point due =
            t0 + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(h_arrival_s[i]));
        while (clk::now() < due) {
            const auto left = due - clk::now();
            if (left > std::chrono::microseconds(200)) std::this_thread::sleep_for(left - std::chrono::microseconds(100));
        }
        for (;;) {
            const tf_status st = tf_serve_submit(s, &reqs[i], &tickets[i]);
            if (st == TF_OK) break;
            if (st != TF_E_BUSY) return st;
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }
    return TF_OK;
}

tf_status tf_serve_report(tf_server *s, tf_serve_stats *out)
{
    if (!s || !out) return TF_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof *out);
    out->completed = (int64_t)s->lat_us.size();
    out->batches = s->batches;
    out->busy_rejects = s->busy_rejects;
    out->max_queue = s->max_queue;
    out->p50_us = percentile(s->lat_us, 0.50);
    out->p90_us = percentile(s->lat_us, 0.90);
    out->p99_us = percentile(s->lat_us, 0.99);
    out->p999_us = percentile(s->lat_us, 0.999);
    double mx = 0.0, sum = 0.0;
    for (double v : s->lat_us) { mx = std::max(mx, v); sum += v; }
    out->max_us = mx;
    out->mean_us = s->lat_us.empty() ? 0.0 : sum / (double)s->lat_us.size();
    const double span = s->have_first ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    out->solves_per_s = span > 0 ? (double)out->completed / span : 0.0;
    out->mean_batch = s->batches ? s->batch_sum / (double)s->batches : 0.0;
    out->failed = s->failed;
    return TF_OK;
}

tf_status tf_serve_reset_stats(tf_server *s)
{
    if (!s) return TF_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->lat_us.clear();
    s->have_first = false;
    s->batches = 0;
    s->busy_rejects = 0;
    s->max_queue = 0;
    s->batch_sum = 0.0;
    s->failed = 0;
    return TF_OK;
}

const char *tf_serve_last_error(tf_server *s)
{
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    thread_local std::string copy;
    copy = s->err;
    return copy.c_str();
}

tf_status tf_serve_inject_fault(tf_server *s, int32_t nbatches)
{
    if (!s || nbatches < 0) return TF_E_INVALID;
    s->inject.store(nbatches);
    return TF_OK;
}

void tf_serve_close(tf_server *s)
{
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->closing = true;
        s->cv_done.wait(lk, [&] {
            if (!s->queue.empty()) return false;
            for (auto &sl : s->slots)
                if (sl->busy) return false;
            return true;
        });
        s->stop = true;
        s->cv_sched.notify_all();
        s->cv_slot.notify_all();
    }
    s->sched.join();
    for (auto &sl : s->slots) sl->completer.join();
    destroy_server(s);
}

// ------------------------------------------------------------------ sync fold-in
tf_status tf_foldin(tf_ctx *ctx, int32_t mode, int32_t nreq, const int64_t *h_req_ptr,
                    const int32_t *d_idx, const double *d_vals, int32_t method, int32_t sweeps,
                    double *d_rows)
{
    if (!ctx) return TF_E_INVALID;
    auto fail = [&](tf_status st, const char *msg) { ctx->err = msg; return st; };
    if (mode < 0 || mode >= ctx->N || nreq < 0 || (nreq > 0 && (!h_req_ptr || !d_rows)))
        return fail(TF_E_INVALID, "bad mode, nreq or NULL pointer");
    if (method != TF_FOLDIN_FULL && method != TF_FOLDIN_CDTF) return fail(TF_E_INVALID, "bad method");
    if (method == TF_FOLDIN_CDTF && sweeps < 1) return fail(TF_E_INVALID, "sweeps must be >= 1");
    if (method == TF_FOLDIN_FULL && ctx->K > kFoldMaxKFull)
        return fail(TF_E_UNSUPPORTED, "full-rank fold-in supports K <= 128");
    if (nreq == 0) return TF_OK;
    if (h_req_ptr[0] != 0) return fail(TF_E_INVALID, "h_req_ptr[0] must be 0");
    for (int32_t q = 0; q < nreq; ++q)
        if (h_req_ptr[q + 1] < h_req_ptr[q]) return fail(TF_E_INVALID, "h_req_ptr must be non-decreasing");
    const int64_t total = h_req_ptr[nreq];
    if (total > 0 && (!d_idx || !d_vals)) return fail(TF_E_INVALID, "NULL entries");
    if (ctx->stale) return fail(TF_E_STATE, "factors were set; call tf_resync first");

    // chunk tables of the full-rank Gram (host), staged with req_ptr
    const bool gram = fold_uses_gram(ctx->K);
    const int64_t nchunks = gram ? fold_chunks(h_req_ptr, nreq) : 0;
    std::vector<int32_t> h_tab((size_t)(nreq + 1 + nchunks));
    if (gram) fold_chunk_tables(h_req_ptr, nreq, h_tab.data(), h_tab.data() + nreq + 1);
    const size_t gs_bytes = (size_t)fold_gram_stride(ctx->K) * ta_bytes(ctx->prec);

    // workspace: req_ptr | chunk tables | P | r | partial Grams | flags
    // (indices, values and rows are the caller's)
    const size_t need = align256((size_t)(nreq + 1) * 8) + align256(h_tab.size() * 4) +
                        align256((size_t)total * ctx->K * ta_bytes(ctx->prec)) +
                        align256((size_t)total * 8) + align256((size_t)nchunks * gs_bytes) + 256;
    void *ws = nullptr;
    if (ctx_alloc(ctx, &ws, need) != hipSuccess) return fail(TF_E_NOMEM, "fold-in workspace");
    char *p = static_cast<char *>(ws);
    int64_t *d_ptr = reinterpret_cast<int64_t *>(p); p += align256((size_t)(nreq + 1) * 8);
    int32_t *d_tab = reinterpret_cast<int32_t *>(p); p += align256(h_tab.size() * 4);
    void *P = p; p += align256((size_t)total * ctx->K * ta_bytes(ctx->prec));
    double *r = reinterpret_cast<double *>(p); p += align256((size_t)total * 8);
    void *gpart = p; p += align256((size_t)nchunks * gs_bytes);
    unsigned long long *flags = reinterpret_cast<unsigned long long *>(p);

    FoldArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = ctx->N; a.mode = mode; a.K = ctx->K; a.nreq = nreq;
    a.req_ptr = d_ptr; a.oidx = d_idx; a.vals = d_vals;
    for (int n = 0; n < ctx->N; ++n) a.A[n] = ctx->m[n].A;
    a.P = P; a.r = r; a.rows = d_rows;
    a.lambda = ctx->lambda; a.reg_mode = ctx->opt.reg_mode; a.sweeps = sweeps;
    a.bad = flags; a.bad_req = flags + 1;
    a.chunk_first = d_tab; a.chunk_req = d_tab + nreq + 1; a.nchunks = (int32_t)nchunks;
    a.gpart = gpart;

    tf_status st = TF_OK;
    unsigned long long hf[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(d_ptr, h_req_ptr, (size_t)(nreq + 1) * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_tab, h_tab.data(), h_tab.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(flags, 0xff, 2 * sizeof(unsigned long long), ctx->stream);
    if (e == hipSuccess) e = launch_fold_validate(a, total, ctx->dims, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && hf[0] != ULLONG_MAX) {
        char buf[128];
        snprintf(buf, sizeof buf, "fold-in entry %llu has a bad index or value", hf[0]);
        ctx->err = buf;
        st = TF_E_INVALID;
    }
    if (e == hipSuccess && st == TF_OK) {
        e = launch_fold_compute(ctx->prec, a, total, method, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess && hf[1] != ULLONG_MAX) {
            char buf[128];
            snprintf(buf, sizeof buf, "fold-in request %llu: non-positive Cholesky pivot (row set to 0)", hf[1]);
            ctx->err = buf;
            st = TF_E_NUMERIC;
        }
    }
    ctx_free(ctx, ws);
    if (e != hipSuccess) {
        ctx->err = std::string("fold-in: ") + hipGetErrorString(e);
        return TF_E_DEVICE;
    }
    return st;
}

}  // extern "C"

// ------------------------------------------------------------------ fold-in without allocation
// tf_foldin_noalloc runs the kernels of tf_foldin with its workspace in one
// file-scope device array per GPU instead of memory it allocates.  In host
// code the array's name is only a stand-in: its device address is looked up
// once per device (fold_scratch_setup, called by tf_init with the device
// current) and only that address is handed to kernels.
namespace {

constexpr size_t kFoldScratchBytes = (size_t)32 << 20;   // per device
constexpr int kScratchDevices = 64;

}  // namespace

static __device__ __align__(256) char scratch[kFoldScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {nullptr};

void *scratch_of(int device)
{
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}

// chunk_first (nreq + 1) and chunk_req of a batch from its entry offsets, by
// one workgroup: per tile of 256 requests, an inclusive scan of the chunk
// counts in LDS, offset by the running total of the earlier tiles.
__global__ __launch_bounds__(256) void k_fold_tables(const int64_t *req_ptr, int32_t nreq,
                                                     int32_t *first, int32_t *req)
{
    __shared__ int32_t sc[256];
    __shared__ int32_t base;
    const int tid = threadIdx.x;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int32_t q0 = 0; q0 < nreq; q0 += 256) {
        const int32_t q = q0 + tid;
        const int32_t cnt = q < nreq
            ? (int32_t)((req_ptr[q + 1] - req_ptr[q] + kFoldChunkEntries - 1) / kFoldChunkEntries) : 0;
        sc[tid] = cnt;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t v = tid >= off ? sc[tid - off] : 0;
            __syncthreads();
            sc[tid] += v;
            __syncthreads();
        }
        const int32_t excl = base + sc[tid] - cnt;
        if (q < nreq) {
            first[q] = excl;
            for (int32_t t = 0; t < cnt; ++t) req[excl + t] = q;
        }
        __syncthreads();
        if (tid == 255) base += sc[255];
        __syncthreads();
    }
    if (tid == 0) first[nreq] = base;
}

// The failure flags start at "none" (a fill kernel rather than a memset).
__global__ void k_fold_flags_init(unsigned long long *flags)
{
    if (threadIdx.x < 2) flags[threadIdx.x] = ~0ull;
}

}  // namespace

namespace tfk {

hipError_t fold_scratch_setup(int device)
{
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

size_t fold_scratch_bytes() { return kFoldScratchBytes; }

}  // namespace tfk

extern "C" tf_status tf_foldin_noalloc(tf_ctx *ctx, int32_t mode, int32_t nreq,
                                       const int64_t *h_req_ptr, const int32_t *d_idx,
                                       const double *d_vals, int32_t method, int32_t sweeps,
                                       double *d_rows)
{
    if (!ctx) return TF_E_INVALID;
    auto fail = [&](tf_status st, const char *msg) { ctx->err = msg; return st; };
    if (mode < 0 || mode >= ctx->N || nreq < 0 || (nreq > 0 && (!h_req_ptr || !d_rows)))
        return fail(TF_E_INVALID, "bad mode, nreq or NULL pointer");
    if (method != TF_FOLDIN_FULL && method != TF_FOLDIN_CDTF) return fail(TF_E_INVALID, "bad method");
    if (method == TF_FOLDIN_CDTF && sweeps < 1) return fail(TF_E_INVALID, "sweeps must be >= 1");
    if (method == TF_FOLDIN_FULL && ctx->K > kFoldMaxKFull)
        return fail(TF_E_UNSUPPORTED, "full-rank fold-in supports K <= 128");
    if (nreq == 0) return TF_OK;
    if (h_req_ptr[0] != 0) return fail(TF_E_INVALID, "h_req_ptr[0] must be 0");
    int64_t nchunks = 0;
    for (int32_t q = 0; q < nreq; ++q) {
        if (h_req_ptr[q + 1] < h_req_ptr[q]) return fail(TF_E_INVALID, "h_req_ptr must be non-decreasing");
        nchunks += (h_req_ptr[q + 1] - h_req_ptr[q] + kFoldChunkEntries - 1) / kFoldChunkEntries;
    }
    const int64_t total = h_req_ptr[nreq];
    if (total > 0 && (!d_idx || !d_vals)) return fail(TF_E_INVALID, "NULL entries");
    if (ctx->stale) return fail(TF_E_STATE, "factors were set; call tf_resync first");
    char *base = static_cast<char *>(scratch_of(ctx->device));
    if (!base) return fail(TF_E_STATE, "no fold-in scratch on this context's device");

    // layout in the scratch array: req_ptr | chunk_first | chunk_req | P | r |
    // partial Grams | flags
    const bool gram = fold_uses_gram(ctx->K);
    if (!gram) nchunks = 0;
    const size_t gs_bytes = (size_t)fold_gram_stride(ctx->K) * ta_bytes(ctx->prec);
    const size_t o_ptr = 0;
    const size_t o_first = o_ptr + align256((size_t)(nreq + 1) * 8);
    const size_t o_creq = o_first + align256((size_t)(nreq + 1) * 4);
    const size_t o_P = o_creq + align256((size_t)nchunks * 4);
    const size_t o_r = o_P + align256((size_t)total * ctx->K * ta_bytes(ctx->prec));
    const size_t o_g = o_r + align256(gram ? 0 : (size_t)total * 8);
    const size_t o_flags = o_g + align256((size_t)nchunks * gs_bytes);
    const size_t need = o_flags + 256;
    if (need > kFoldScratchBytes) {
        char buf[160];
        snprintf(buf, sizeof buf, "fold-in batch needs %zu bytes of workspace; the scratch holds %zu",
                 need, kFoldScratchBytes);
        return fail(TF_E_INVALID, buf);
    }
    int64_t *d_ptr = reinterpret_cast<int64_t *>(base + o_ptr);
    unsigned long long *flags = reinterpret_cast<unsigned long long *>(base + o_flags);

    FoldArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = ctx->N; a.mode = mode; a.K = ctx->K; a.nreq = nreq;
    a.req_ptr = d_ptr; a.oidx = d_idx; a.vals = d_vals;
    for (int n = 0; n < ctx->N; ++n) a.A[n] = ctx->m[n].A;
    a.P = base + o_P;
    a.r = gram ? nullptr : reinterpret_cast<double *>(base + o_r);
    a.rows = d_rows;
    a.lambda = ctx->lambda; a.reg_mode = ctx->opt.reg_mode; a.sweeps = sweeps;
    a.bad = flags; a.bad_req = flags + 1;
    a.chunk_first = reinterpret_cast<int32_t *>(base + o_first);
    a.chunk_req = reinterpret_cast<int32_t *>(base + o_creq);
    a.nchunks = (int32_t)nchunks;
    a.gpart = base + o_g;

    tf_status st = TF_OK;
    unsigned long long hf[2] = {0, 0};
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(d_ptr, h_req_ptr, (size_t)(nreq + 1) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && gram) {
        hipLaunchKernelGGL(k_fold_tables, dim3(1), dim3(256), 0, s, d_ptr, nreq,
                           reinterpret_cast<int32_t *>(base + o_first),
                           reinterpret_cast<int32_t *>(base + o_creq));
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fold_flags_init, dim3(1), dim3(64), 0, s, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_fold_validate(a, total, ctx->dims, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && hf[0] != ULLONG_MAX) {
        char buf[128];
        snprintf(buf, sizeof buf, "fold-in entry %llu has a bad index or value", hf[0]);
        ctx->err = buf;
        st = TF_E_INVALID;
    }
    if (e == hipSuccess && st == TF_OK) {
        e = launch_fold_compute(ctx->prec, a, total, method, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && hf[1] != ULLONG_MAX) {
            char buf[128];
            snprintf(buf, sizeof buf, "fold-in request %llu: non-positive Cholesky pivot (row set to 0)", hf[1]);
            ctx->err = buf;
            st = TF_E_NUMERIC;
        }
    }
    if (e != hipSuccess) {
        char buf[160];
        snprintf(buf, sizeof buf, "fold-in: %s", hipGetErrorString(e));
        ctx->err = buf;
        return TF_E_DEVICE;
    }
    return st;
}
