// Continuous-batching QIEO server.
//
// Requests (a knapsack problem plus a generation budget) are submitted from
// any thread.  A worker thread owns one multi-instance engine over a device
// pool whose size is the HBM budget.  Each iteration it
//   1. admits queued requests in arrival order while the pool has room for
//      their populations (and the resident count is under the cap),
//   2. advances every resident population by min(G, remaining) generations
//      in the same fused launches (graph-replayed),
//   3. retires populations whose budget is spent: reads their best-so-far
//      record, frees their memory, stamps the completion time.
// A request is processed exactly as qieo_step would process it alone, so its
// result does not depend on what else was resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qieo.h"
#include "qieo_multi.hpp"

using namespace qieo;

namespace {

using clock_type = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    std::vector<qieo_item> items;
    int32_t capacity = 0, n_pop = 0, n_gen = 0;
    uint64_t seed = 0;
    clock_type::time_point arrival, admitted, completed;
    int32_t remaining = 0;
    int status = QIEO_EAGAIN;          // QIEO_OK when done, an error code on failure
    qieo_result result{};
    std::vector<uint32_t> bits;
    size_t bytes = 0;                  // device footprint
};

}  // namespace

struct qieo_server {
    qieo_server_cfg cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    DevicePool pool;
    Engine* eng = nullptr;

    std::mutex mu;
    std::condition_variable cv_work;   // worker waits for submissions
    std::condition_variable cv_done;   // callers wait for completions
    std::deque<Request*> queue;        // submitted, not yet admitted (FIFO)
    std::vector<Request*> resident;    // parallel to the engine's members
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool onchip = true;                // batched on-chip loop (the worker applies it)
    int worker_error = QIEO_OK;
    std::string worker_msg;

    // statistics (under mu)
    int64_t iterations = 0, admitted = 0, completed = 0, failed = 0;
    double gene_updates = 0.0;
    size_t peak_resident = 0, peak_pool = 0;

    std::thread worker;
};

static void server_loop(qieo_server* s)
{
    (void)hipSetDevice(s->device);
    std::vector<int32_t> gens;
    bool onchip = !s->onchip;          // applied below on the first pass
    for (;;) {
        std::vector<Request*> to_admit;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->resident.empty(); });
            if (s->stop) return;
            // the engine is the worker's alone: a change of mode reaches it here
            if (s->onchip != onchip) {
                onchip = s->onchip;
                s->eng->set_use_onchip(onchip);
            }
            // admission in arrival order, limited by the resident cap; memory is
            // checked below, where the allocation itself is attempted
            size_t cap = s->cfg.max_resident > 0 ? (size_t)s->cfg.max_resident : (size_t)-1;
            while (!s->queue.empty() && s->resident.size() + to_admit.size() < cap) {
                to_admit.push_back(s->queue.front());
                s->queue.pop_front();
            }
        }
        std::vector<Request*> back;   // not admitted this time: return to the queue head
        bool blocked = false;
        for (Request* r : to_admit) {
            if (blocked) { back.push_back(r); continue; }
            if (r->bytes > s->pool.capacity()) {
                std::lock_guard<std::mutex> lk(s->mu);
                r->status = QIEO_ENOMEM;
                r->completed = clock_type::now();
                s->failed++;
                s->cv_done.notify_all();
                continue;
            }
            int rc = s->eng->add(s->pool, r->items.data(), (int32_t)r->items.size(), r->capacity,
                                 r->n_pop, r->seed, r->ticket, s->cfg.convergence_window);
            if (rc == QIEO_ENOMEM) {
                blocked = true;        // head of line waits for memory to free up
                back.push_back(r);
                continue;
            }
            std::lock_guard<std::mutex> lk(s->mu);
            if (rc != QIEO_OK) {
                r->status = rc;
                r->completed = clock_type::now();
                s->failed++;
                s->cv_done.notify_all();
                continue;
            }
            r->admitted = clock_type::now();
            r->remaining = r->n_gen;
            r->items.clear();
            r->items.shrink_to_fit();
            s->resident.push_back(r);
            s->admitted++;
        }
        if (!back.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto it = back.rbegin(); it != back.rend(); ++it) s->queue.push_front(*it);
        }
        if (s->resident.empty()) {
            if (blocked) {
                // nothing resident yet no room: cannot happen unless the pool is
                // fragmented beyond use; fail the head request to make progress
                std::lock_guard<std::mutex> lk(s->mu);
                if (!s->queue.empty()) {
                    Request* r = s->queue.front();
                    s->queue.pop_front();
                    r->status = QIEO_ENOMEM;
                    r->completed = clock_type::now();
                    s->failed++;
                    s->cv_done.notify_all();
                }
            }
            continue;
        }
        // advance every resident population
        const int G = s->cfg.gens_per_iter > 0 ? s->cfg.gens_per_iter : 25;
        gens.resize(s->resident.size());
        double work = 0.0;
        for (size_t i = 0; i < s->resident.size(); ++i) {
            gens[i] = std::min<int32_t>(G, s->resident[i]->remaining);
            const Member& m = s->eng->member(i);
            work += (double)gens[i] * m.np * m.ng;
        }
        int rc = s->eng->run(gens.data());
        if (rc == QIEO_OK) rc = s->eng->sync();
        if (rc == QIEO_OK && s->cfg.convergence_window > 0) rc = s->eng->refresh_status();
        if (rc != QIEO_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->worker_error = rc;
            s->worker_msg = qieo_last_error();
            for (Request* r : s->resident) {
                r->status = rc;
                r->completed = clock_type::now();
            }
            s->resident.clear();
            s->stop = true;
            s->cv_done.notify_all();
            return;
        }
        // retire finished populations (highest index first keeps indices valid)
        std::vector<size_t> done;
        for (size_t i = 0; i < s->resident.size(); ++i) {
            s->resident[i]->remaining -= gens[i];
            const bool conv = s->cfg.convergence_window > 0 && s->eng->member(i).converged;
            if (s->resident[i]->remaining == 0 || conv) done.push_back(i);
        }
        for (size_t k = done.size(); k-- > 0;) {
            const size_t i = done[k];
            Request* r = s->resident[i];
            Member& m = s->eng->member(i);
            r->bits.assign(((size_t)m.ng + 31) / 32, 0u);
            const int rr = read_best(m.d, m.capacity, s->stream, &r->result, r->bits.data(),
                                     r->bits.size());
            const auto now = clock_type::now();
            s->eng->remove_at(i, s->pool);
            std::lock_guard<std::mutex> lk(s->mu);
            s->resident.erase(s->resident.begin() + i);
            r->status = rr;
            r->completed = now;
            s->completed++;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->iterations++;
        s->gene_updates += work;
        s->peak_resident = std::max(s->peak_resident, s->resident.size());
        s->peak_pool = std::max(s->peak_pool, s->pool.used());
        if (!done.empty()) s->cv_done.notify_all();
    }
}

static void server_release(qieo_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    delete s->eng;
    for (auto& kv : s->all) delete kv.second;
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

extern "C" int qieo_server_create(const qieo_server_cfg* cfg, const qieo_dev_ctx* ctx,
                                  qieo_server** out)
{
    clear_error();
    if (!out || !cfg) return set_error(QIEO_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->hbm_budget_bytes < 4096)
        return set_error(QIEO_EINVAL, "hbm_budget_bytes too small (%zu)", cfg->hbm_budget_bytes);
    if (cfg->max_resident < 0 || cfg->gens_per_iter < 0)
        return set_error(QIEO_EINVAL, "max_resident and gens_per_iter must be >= 0");
    if (cfg->convergence_window < 0 || cfg->convergence_window > kConvRing)
        return set_error(QIEO_EINVAL, "convergence_window must be in [0, %d]", kConvRing);
    if (ctx && ((ctx->alloc == nullptr) != (ctx->free == nullptr)))
        return set_error(QIEO_EINVAL, "ctx->alloc and ctx->free must be both set or both NULL");
    int rc = check_device();
    if (rc) return rc;
    qieo_server* s = new (std::nothrow) qieo_server();
    if (!s) return set_error(QIEO_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    hipError_t e;
    if (ctx && ctx->stream) {
        s->stream = (hipStream_t)ctx->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
            server_release(s);
            return rc;
        }
        s->own_stream = true;
    }
    if ((rc = s->pool.init(cfg->hbm_budget_bytes, ctx))) {
        server_release(s);
        return rc;
    }
    s->eng = new (std::nothrow) Engine(s->stream, ctx);
    if (!s->eng) {
        server_release(s);
        return set_error(QIEO_ENOMEM, "host allocation failed");
    }
    // Membership changes nearly every iteration here and each change
    // rebuilds the segment table, so only the >= 32-chunk rows take segment
    // order (20,000 requests at 500/s: 376.4 s with the 8-31-chunk rows
    // merged into the table, 373.8-374.9 s without).
    s->eng->set_use_segments(2);
    s->worker = std::thread(server_loop, s);
    *out = s;
    return QIEO_OK;
}

extern "C" int qieo_server_set_onchip(qieo_server* s, int32_t enabled)
{
    clear_error();
    if (!s) return set_error(QIEO_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->onchip = enabled != 0;
    return QIEO_OK;
}

extern "C" int qieo_server_submit(qieo_server* s, const qieo_problem* p, int32_t n_gen,
                                  uint64_t* ticket)
{
    clear_error();
    if (!s || !p || !ticket) return set_error(QIEO_EINVAL, "NULL argument");
    if (n_gen < 1) return set_error(QIEO_EINVAL, "n_gen must be >= 1 (got %d)", n_gen);
    int rc = validate_problem(p->items, p->n_items, p->capacity, p->n_pop);
    if (rc) return rc;
    Request* r = new (std::nothrow) Request();
    if (!r) return set_error(QIEO_ENOMEM, "host allocation failed");
    r->arrival = clock_type::now();
    try {
        r->items.assign(p->items, p->items + p->n_items);
    } catch (...) {
        delete r;
        return set_error(QIEO_ENOMEM, "host allocation failed");
    }
    r->capacity = p->capacity;
    r->n_pop = p->n_pop;
    r->n_gen = n_gen;
    r->seed = p->seed;
    ArenaLayout L;
    r->bytes = arena_layout(p->n_items, p->n_pop, &L);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return set_error(s->worker_error ? s->worker_error : QIEO_ESTATE,
                             "server is stopped: %s", s->worker_msg.c_str());
        }
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return QIEO_OK;
}

static int fill_result(Request* r, qieo_result* out, uint32_t* bits, size_t n_words,
                       int64_t* latency_ns)
{
    if (r->status != QIEO_OK) return set_error(r->status, "request %llu failed: %s",
                                               (unsigned long long)r->ticket,
                                               qieo_strerror(r->status));
    if (bits && n_words < r->bits.size())
        return set_error(QIEO_EINVAL, "bits buffer has %zu words, needs %zu", n_words,
                         r->bits.size());
    if (out) *out = r->result;
    if (bits) std::memcpy(bits, r->bits.data(), r->bits.size() * sizeof(uint32_t));
    if (latency_ns)
        *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(r->completed - r->arrival)
                          .count();
    return QIEO_OK;
}

extern "C" int qieo_server_poll(qieo_server* s, uint64_t ticket, qieo_result* out,
                                uint32_t* bits, size_t n_words, int64_t* latency_ns)
{
    clear_error();
    if (!s) return set_error(QIEO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(QIEO_EINVAL, "unknown ticket %llu",
                                             (unsigned long long)ticket);
    Request* r = it->second;
    if (r->status == QIEO_EAGAIN) return QIEO_EAGAIN;
    return fill_result(r, out, bits, n_words, latency_ns);
}

extern "C" int qieo_server_wait(qieo_server* s, uint64_t ticket, qieo_result* out,
                                uint32_t* bits, size_t n_words, int64_t* latency_ns)
{
    clear_error();
    if (!s) return set_error(QIEO_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(QIEO_EINVAL, "unknown ticket %llu",
                                             (unsigned long long)ticket);
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->status != QIEO_EAGAIN || (s->stop && s->worker_error); });
    if (r->status == QIEO_EAGAIN) return set_error(s->worker_error, "server stopped: %s",
                                                   s->worker_msg.c_str());
    return fill_result(r, out, bits, n_words, latency_ns);
}

extern "C" int qieo_server_release(qieo_server* s, uint64_t ticket)
{
    clear_error();
    if (!s) return set_error(QIEO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(QIEO_EINVAL, "unknown ticket %llu",
                                             (unsigned long long)ticket);
    if (it->second->status == QIEO_EAGAIN)
        return set_error(QIEO_ESTATE, "request %llu is not finished",
                         (unsigned long long)ticket);
    delete it->second;
    s->all.erase(it);
    return QIEO_OK;
}

extern "C" int qieo_server_get_stats(qieo_server* s, qieo_server_stats* st)
{
    clear_error();
    if (!s || !st) return set_error(QIEO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->queued = (int64_t)s->queue.size();
    st->resident = (int64_t)s->resident.size();
    st->admitted = s->admitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->iterations = s->iterations;
    st->gene_updates = s->gene_updates;
    st->pool_bytes = s->pool.capacity();
    st->pool_used = s->pool.used();
    st->peak_resident = (int64_t)s->peak_resident;
    st->peak_pool_used = s->peak_pool;
    st->error = s->worker_error;
    return QIEO_OK;
}

extern "C" void qieo_server_destroy(qieo_server* s) { server_release(s); }
