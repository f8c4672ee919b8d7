// libqieo host runtime: C ABI, validation, device memory, streams, timing.
//
// One instance owns one device arena (a single allocation, carved into the
// planes described in qieo_kernels.hpp) and one stream.  qieo_step enqueues
// one fused generation launch per generation plus one finishing launch, all
// on that stream; nothing crosses back to the host inside the loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qieo.h"
#include "qieo_internal.hpp"
#include "qieo_kernels.hpp"
#include "qieo_onchip.hpp"

using namespace qieo;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
namespace qieo {

int hip_fail(hipError_t e, const char* what)
{
    return set_error(QIEO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void* DevMem::alloc(size_t bytes) const
{
    if (custom) return ctx.alloc(bytes, ctx.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void DevMem::release(void* p) const
{
    if (!p) return;
    if (custom) ctx.free(p, ctx.user);
    else (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// Device arena
// ---------------------------------------------------------------------------
InstDev bind_arena(char* base, const ArenaLayout& L, int32_t ng, int32_t np, int32_t cap,
                   uint64_t seed)
{
    InstDev d{};
    d.alpha = reinterpret_cast<float*>(base + L.alpha);
    d.beta = reinterpret_cast<float*>(base + L.beta);
    d.xbits = reinterpret_cast<uint32_t*>(base + L.xbits);
    d.v = reinterpret_cast<const int32_t*>(base + L.v);
    d.w = reinterpret_cast<const int32_t*>(base + L.w);
    d.fit = reinterpret_cast<int32_t*>(base + L.fit);
    d.prof = reinterpret_cast<int32_t*>(base + L.prof);
    d.wt = reinterpret_cast<int32_t*>(base + L.wt);
    d.ekey = reinterpret_cast<unsigned long long*>(base + L.ekey);
    d.best = reinterpret_cast<int32_t*>(base + L.best);
    d.best_bits = reinterpret_cast<uint32_t*>(base + L.best_bits);
    d.tbase = reinterpret_cast<int64_t*>(base + L.tbase);
    d.conv = reinterpret_cast<int32_t*>(base + L.conv);
    d.part = reinterpret_cast<uint32_t*>(base + L.part);
    d.sync = reinterpret_cast<uint32_t*>(base + L.sync);
    d.np = np;
    d.ng = ng;
    d.pitch = L.pitch;
    d.nchunk = L.nchunk;
    d.capacity = cap;
    d.seed_lo = (uint32_t)seed;
    d.seed_hi = (uint32_t)(seed >> 32);
    return d;
}

// Upload item tables (zero-padded to pitch) and initialise the state.
int upload_and_init(const InstDev& d, const qieo_item* items, hipStream_t s,
                    const ArenaLayout& L, char* base, std::vector<int32_t>& staging, bool f64)
{
    const size_t pitch = (size_t)d.nchunk * kChunk;   // v, w are zero-padded to whole chunks
    staging.assign(2 * pitch, 0);
    for (int32_t i = 0; i < d.ng; ++i) {
        staging[i] = items[i].profit;
        staging[pitch + i] = items[i].weight;
    }
    hipError_t e;
    if ((e = hipMemsetAsync(base + L.zero_from, 0, L.total - L.zero_from, s)) != hipSuccess)
        return hip_fail(e, "hipMemsetAsync");
    if ((e = hipMemcpyAsync(base + L.v, staging.data(), pitch * sizeof(int32_t),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(v)");
    if ((e = hipMemcpyAsync(base + L.w, staging.data() + pitch, pitch * sizeof(int32_t),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(w)");
    if ((e = launch_init(d, s, f64)) != hipSuccess) return hip_fail(e, "init kernel");
    return QIEO_OK;
}

int check_device()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t p;
    if ((e = hipGetDeviceProperties(&p, dev)) != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return set_error(QIEO_EDEVICE, "device %d is %s, libqieo is built for gfx950", dev,
                         p.gcnArchName);
    return QIEO_OK;
}

}  // namespace qieo

// ---------------------------------------------------------------------------
// Single instance
// ---------------------------------------------------------------------------
struct qieo_inst {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevMem mem;                  // the caller's allocator, or hipMalloc
    char* arena = nullptr;
    ArenaLayout L{};
    InstDev d{};
    InstDev* d_desc = nullptr;   // device copy of the descriptor (inside its own alloc)
    InstDev* h_desc = nullptr;   // pinned host staging of the descriptor
    int32_t ng = 0, np = 0, capacity = 0;
    uint64_t seed = 0;
    uint64_t items_hash = 0;     // FNV-1a of the item array (checkpoint identity)
    int64_t t = 0;               // generations enqueued so far
    int R = 1, S = 1, flags = 0;
    int pipeline = QIEO_PIPELINE_FUSED;
    bool f64 = false;            // binary64 amplitudes
    int persistent = 1;          // see qieo_set_persistent
    bool onchip_check = false;   // an on-chip launch is queued: qieo_sync reads its abort flag
    bool items_packed = false;   // profits and weights fit the on-chip loop's packed item tables
    int32_t last_path = -1;      // QIEO_PATH_* of the last step call
    int64_t barrier_us = 1000000;    // bound on one on-chip grid-barrier wait
    bool use_graph = true;       // replay a captured graph of a call's launches
    hipGraphExec_t graph = nullptr;
    int32_t graph_n = -1;        // generations the cached graph runs
    int graph_key = -1;          // shape/variant it was captured with
    int32_t prev_n = -1;         // generations and shape/variant of the previous
    int prev_key = -1;           // fused call (capture starts on a repeat)
    int32_t window = 0;
    int32_t* h_fit = nullptr;                // pinned, host DetermineElite
    unsigned long long* h_key = nullptr;     // pinned, host DetermineElite
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop) per timed launch
    std::vector<int> ev_stage;   // stage of each pair
    size_t ev_used = 0;
    int64_t launches[kStages] = {0, 0, 0, 0, 0};
    double total_ms[kStages] = {0, 0, 0, 0, 0};
};

static void inst_release(qieo_inst* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->h_fit) (void)hipHostFree(h->h_fit);
    if (h->h_key) (void)hipHostFree(h->h_key);
    h->mem.release(h->arena);
    h->mem.release(h->d_desc);
    if (h->h_desc) (void)hipHostFree(h->h_desc);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

// The handle's work shape when the caller sets none: the tuning database's
// entry for its bucket, else the built-in rule.  Binary64 amplitudes: in
// segment order with non-temporal loads and stores when streaming (its
// transfers go through LDS as whole 1 KB lines); otherwise row order with at
// most 2 rows and 4 waves per workgroup (twice the registers per gene),
// prefetch and cached loads (the row kernel's 32-byte-per-lane non-temporal
// loads were slower in every binary64 shape measured).
static void default_shape(const qieo_inst* h, int* R, int* S, int* F)
{
    if (h->f64 || !tuned_tile(h->np, h->L.nchunk, R, S, F))
        pick_tile(h->np, h->L.nchunk, R, S, F, h->f64 ? 8 : 4);
    if (h->f64) {
        *R = std::min(*R, 2);
        *S = std::min(*S, 4);
        const int64_t planes = (int64_t)h->np * h->L.nchunk * kChunk * 2 * 8;
        if (planes > ((int64_t)256 << 20))
            // 4.42 ms per generation at 4096 x 200,000 against 5.76 in row order
            *F = kFlagSegments | kFlagNontemporal | kFlagNontemporalLoads;
        else
            *F = (*F & ~(kFlagNontemporalLoads | kFlagPrefetch | kFlagSegments)) |
                 (h->L.nchunk > *S ? kFlagPrefetch : 0);
    }
}

static int create_impl(const qieo_item* items, int32_t n_items, int32_t capacity,
                       int32_t n_pop, uint64_t seed, const qieo_dev_ctx* ctx, bool f64,
                       qieo_inst** out)
{
    clear_error();
    if (!out) return set_error(QIEO_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_problem(items, n_items, capacity, n_pop);
    if (rc) return rc;
    if (ctx && ((ctx->alloc == nullptr) != (ctx->free == nullptr)))
        return set_error(QIEO_EINVAL, "ctx->alloc and ctx->free must be both set or both NULL");
    if ((rc = check_device())) return rc;

    qieo_inst* h = new (std::nothrow) qieo_inst();
    if (!h) return set_error(QIEO_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&h->device);
    h->mem.set(ctx);
    hipError_t e;
    if (ctx && ctx->stream) {
        h->stream = (hipStream_t)ctx->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
            inst_release(h);
            return rc;
        }
        h->own_stream = true;
    }
    h->ng = n_items;
    h->np = n_pop;
    h->items_packed = items_packable(items, n_items);
    h->capacity = capacity;
    h->seed = seed;
    h->items_hash = items_fnv1a(items, n_items);
    h->f64 = f64;
    arena_layout(n_items, n_pop, &h->L, f64 ? 8 : 4);
    h->arena = (char*)h->mem.alloc(h->L.total);
    h->d_desc = h->arena ? (InstDev*)h->mem.alloc(sizeof(InstDev)) : nullptr;
    if (!h->arena || !h->d_desc) {
        inst_release(h);
        return set_error(QIEO_ENOMEM, "device allocation of %zu bytes failed", h->L.total);
    }
    if ((e = hipHostMalloc((void**)&h->h_desc, sizeof(InstDev), hipHostMallocDefault)) !=
        hipSuccess) {
        rc = hip_fail(e, "hipHostMalloc");
        inst_release(h);
        return rc;
    }
    h->d = bind_arena(h->arena, h->L, n_items, n_pop, capacity, seed);
    std::vector<int32_t> staging;
    if ((rc = upload_and_init(h->d, items, h->stream, h->L, h->arena, staging, f64))) {
        inst_release(h);
        return rc;
    }
    *h->h_desc = h->d;
    if ((e = hipMemcpyAsync(h->d_desc, h->h_desc, sizeof(InstDev), hipMemcpyHostToDevice,
                            h->stream)) != hipSuccess) {
        rc = hip_fail(e, "hipMemcpyAsync(descriptor)");
        inst_release(h);
        return rc;
    }
    default_shape(h, &h->R, &h->S, &h->flags);
    if (f64) h->persistent = 0;
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) {
        rc = hip_fail(e, "hipStreamSynchronize");
        inst_release(h);
        return rc;
    }
    *out = h;
    return QIEO_OK;
}

extern "C" int qieo_create_ex(const qieo_item* items, int32_t n_items, int32_t capacity,
                              int32_t n_pop, uint64_t seed, const qieo_dev_ctx* ctx,
                              qieo_inst** out)
{
    return create_impl(items, n_items, capacity, n_pop, seed, ctx, false, out);
}

extern "C" int qieo_create_f64(const qieo_item* items, int32_t n_items, int32_t capacity,
                               int32_t n_pop, uint64_t seed, const qieo_dev_ctx* ctx,
                               qieo_inst** out)
{
    return create_impl(items, n_items, capacity, n_pop, seed, ctx, true, out);
}

extern "C" int qieo_create(const qieo_item* items, int32_t n_items, int32_t capacity,
                           int32_t n_pop, uint64_t seed, qieo_inst** out)
{
    return create_impl(items, n_items, capacity, n_pop, seed, nullptr, false, out);
}

static int timed_event_pair(qieo_inst* h, int stage, hipEvent_t* a, hipEvent_t* b)
{
    while (h->ev.size() < 2 * (h->ev_used + 1)) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
        h->ev.push_back(e);
    }
    if (h->ev_stage.size() < h->ev_used + 1) h->ev_stage.resize(h->ev_used + 1);
    h->ev_stage[h->ev_used] = stage;
    *a = h->ev[2 * h->ev_used];
    *b = h->ev[2 * h->ev_used + 1];
    h->ev_used++;
    return QIEO_OK;
}

static int collect_timing(qieo_inst* h)
{
    if (h->ev_used == 0) return QIEO_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (size_t k = 0; k < h->ev_used; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        h->total_ms[h->ev_stage[k]] += ms;
        h->launches[h->ev_stage[k]]++;
    }
    h->ev_used = 0;
    return QIEO_OK;
}

// Host DetermineElite of the unfused pipeline: fitness to the host, argmax
// (lowest row on ties), elite key back to the device.
static int host_elite(qieo_inst* h, int64_t t)
{
    hipError_t e;
    const int par = (int)(t & 1);
    if ((e = hipMemcpyAsync(h->h_fit, h->d.fit + (size_t)par * h->np, h->np * sizeof(int32_t),
                            hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(fitness)");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return hip_fail(e, "hipStreamSynchronize");
    int32_t best = 0;
    for (int32_t c = 1; c < h->np; ++c)
        if (h->h_fit[c] > h->h_fit[best]) best = c;
    *h->h_key = ((unsigned long long)((uint32_t)h->h_fit[best] ^ 0x80000000u) << 32) |
                (unsigned long long)(~(uint32_t)best);
    if ((e = hipMemcpyAsync(h->d.ekey + t % 3, h->h_key, sizeof(unsigned long long),
                            hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(elite)");
    return QIEO_OK;
}

// Generation k of a call of n on the fused path: the row kernel with the
// handle's work shape, or the segment-order launches.
static hipError_t launch_fused(qieo_inst* h, int blocks, int k, int n)
{
    if (h->flags & kFlagSegments)
        return launch_segments(h->d_desc, h->np, h->L.nchunk, h->L.part_nseg, h->flags, k, n,
                               h->f64, h->stream);
    return launch_generation(h->d_desc, nullptr, blocks, h->R, h->S, h->flags, k, nullptr, n,
                             h->stream);
}

// Captures the n fused launches of one call (and the finishing launch) into
// h->graph.  Relaxed mode: the sequence holds kernel launches only.  If the
// capture does not complete (another thread's device-wide call can
// invalidate a capture in progress), h->graph stays NULL and the caller
// enqueues the same launches directly; the error state is left clear.
static void capture_call(qieo_inst* h, int32_t n, int blocks)
{
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    h->graph_n = -1;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipError_t le = hipSuccess;
    for (int32_t k = 0; k < n && le == hipSuccess; ++k)
        le = launch_fused(h, blocks, k, n);
    if (le == hipSuccess) le = launch_finish(h->d_desc, 1, nullptr, n, nullptr, h->stream);
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    hipGraphExec_t x = nullptr;
    if (le == hipSuccess && e == hipSuccess && g &&
        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
        h->graph = x;
        h->graph_n = n;
        h->graph_key = (h->R * 32 + h->S) * 32 + h->flags;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
}

extern "C" int qieo_step_async(qieo_inst* h, int32_t n)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (n < 0) return set_error(QIEO_EINVAL, "n_generations must be >= 0 (got %d)", n);
    if (n == 0) return QIEO_OK;
    if (h->t + n > (int64_t)INT32_MAX)
        return set_error(QIEO_EINVAL, "generation index would exceed 2^31-1");
    hipError_t e;
    const int blocks = (h->np + h->R - 1) / h->R;
    if (h->f64) {
        h->last_path = QIEO_PATH_LAUNCHES;
        for (int32_t k = 0; k < n; ++k) {
            hipEvent_t a = nullptr, b = nullptr;
            if (h->timing) {
                int rc = timed_event_pair(h, 0, &a, &b);
                if (rc) return rc;
                (void)hipEventRecord(a, h->stream);
            }
            e = (h->flags & kFlagSegments)
                    ? launch_segments(h->d_desc, h->np, h->L.nchunk, h->L.part_nseg, h->flags,
                                      k, n, true, h->stream)
                    : launch_generation_f64(h->d_desc, blocks, h->R, h->S, h->flags, k, n,
                                            h->stream);
            if (e != hipSuccess) return hip_fail(e, "generation kernel (binary64)");
            if (h->timing) (void)hipEventRecord(b, h->stream);
        }
        if ((e = launch_finish(h->d_desc, 1, nullptr, n, nullptr, h->stream)) != hipSuccess)
            return hip_fail(e, "finish kernel");
        h->t += n;
        return QIEO_OK;
    }
    // populations whose planes fit the chip's registers: the whole call in
    // one cooperative launch that holds them there (mode 1 from
    // kOnchipMinGens generations on, where the planes' one load and one store
    // per call cost less than the per-generation launches' traffic, for
    // populations large enough to pay for its synchronisation; mode 3 for
    // every call), with or without a convergence window.
    if (h->pipeline == QIEO_PIPELINE_FUSED &&
        (h->persistent == 3 || (h->persistent == 1 && n >= kOnchipMinGens &&
                                onchip_worth(h->np, h->L.nchunk)))) {
        OnchipPlan p;
        size_t lim = 0;
        int ncu = 0;
        onchip_limits(&lim, &ncu);
        if (ncu > 0 && onchip_plan(h->np, h->L.nchunk, ncu, lim, &p, h->items_packed)) {
            hipEvent_t a = nullptr, b = nullptr;
            if (h->timing) {
                int rc = timed_event_pair(h, 0, &a, &b);
                if (rc) return rc;
                (void)hipEventRecord(a, h->stream);
            }
            p.conv = h->window > 0;
            if ((e = launch_onchip(h->d_desc, p, n, onchip_spin_ticks(h->device, h->barrier_us),
                                   h->stream)) !=
                hipSuccess)
                return hip_fail(e, "on-chip kernel");
            h->onchip_check = true;
            h->last_path = QIEO_PATH_ONCHIP;
            if (h->timing) (void)hipEventRecord(b, h->stream);
            if ((e = launch_finish(h->d_desc, 1, nullptr, n, nullptr, h->stream)) != hipSuccess)
                return hip_fail(e, "finish kernel");
            h->t += n;
            return QIEO_OK;
        }
    }
    // small populations: the whole call in one single-workgroup launch, from
    // LDS when the whole state fits there.  Mode 1 takes it only where it
    // measured faster than launches: at most one (row, chunk) item per wave,
    // since a wave's items run one after another, each a long dependent chain
    // (2.5 us), while launches spread them over the whole chip.
    const size_t lds = resident_lds_bytes(h->np, h->L.pitch, h->L.nchunk);
    const int64_t items = (int64_t)h->np * h->L.nchunk;
    const bool fits_lds = (h->persistent == 2 || (h->persistent == 1 && items <= 16)) &&
                          lds <= resident_lds_limit();
    if (h->pipeline == QIEO_PIPELINE_FUSED &&
        (fits_lds || (h->persistent == 2 && h->np <= kPersistentMaxRows))) {
        hipEvent_t a = nullptr, b = nullptr;
        if (h->timing) {
            int rc = timed_event_pair(h, 0, &a, &b);
            if (rc) return rc;
            (void)hipEventRecord(a, h->stream);
        }
        const int waves = (int)std::min<int64_t>(16, (int64_t)h->np * h->L.nchunk);
        e = fits_lds ? launch_resident(h->d_desc, nullptr, 1, waves, lds, nullptr, n, h->stream)
                     : launch_persistent(h->d_desc, nullptr, 1, waves, nullptr, n, h->stream);
        if (e != hipSuccess) return hip_fail(e, "persistent kernel");
        h->last_path = fits_lds ? QIEO_PATH_LDS : QIEO_PATH_GLOBAL;
        if (h->timing) (void)hipEventRecord(b, h->stream);
        if ((e = launch_finish(h->d_desc, 1, nullptr, n, nullptr, h->stream)) != hipSuccess)
            return hip_fail(e, "finish kernel");
        h->t += n;
        return QIEO_OK;
    }
    h->last_path = QIEO_PATH_LAUNCHES;
    // fused per-generation launches: replay one captured graph per call.  A
    // call is captured once it repeats (same generation count, same shape and
    // variant as the previous call): capturing a one-off call costs more than
    // launching it.
    if (h->pipeline == QIEO_PIPELINE_FUSED && h->use_graph && !h->timing && n >= 2) {
        const int key = (h->R * 32 + h->S) * 32 + h->flags;
        const bool cached = h->graph && h->graph_n == n && h->graph_key == key;
        const bool repeat = h->prev_n == n && h->prev_key == key;
        h->prev_n = n;
        h->prev_key = key;
        if (!cached && repeat) capture_call(h, n, blocks);
        if (h->graph && h->graph_n == n && h->graph_key == key) {
            if ((e = hipGraphLaunch(h->graph, h->stream)) != hipSuccess)
                return hip_fail(e, "hipGraphLaunch");
            h->t += n;
            return QIEO_OK;
        }
        // no graph (the capture was lost): the same launches, enqueued directly
    }
    // stage list of one generation
    int stages[4], nst = 0;
    if (h->pipeline == QIEO_PIPELINE_FUSED) {
        stages[nst++] = kStepAll;
    } else if (h->pipeline == QIEO_PIPELINE_CHROMOSOME) {
        stages[nst++] = -2;
    } else {
        stages[nst++] = kStepCip;
        stages[nst++] = kStepQip;
        stages[nst++] = h->pipeline == QIEO_PIPELINE_UNFUSED_FE_DE ? (kStepFe | kStepDe) : kStepFe;
        if (h->pipeline == QIEO_PIPELINE_UNFUSED) stages[nst++] = kStepDe;
        if (h->pipeline == QIEO_PIPELINE_UNFUSED_HOST_DE) stages[nst++] = -1;   // host
    }
    for (int32_t k = 0; k < n; ++k) {
        for (int si = 0; si < nst; ++si) {
            const int st = stages[si];
            const int slot = (st == kStepAll || st == -2) ? 0 : st == kStepCip ? 1
                           : st == kStepQip ? 2 : (st > 0 && (st & kStepFe)) ? 3 : 4;
            hipEvent_t a = nullptr, b = nullptr;
            if (h->timing) {
                int rc = timed_event_pair(h, slot, &a, &b);
                if (rc) return rc;
                (void)hipEventRecord(a, h->stream);
            }
            if (st == kStepAll) {
                if ((e = launch_fused(h, blocks, k, n)) != hipSuccess)
                    return hip_fail(e, "generation kernel");
            } else if (st == -1) {
                int rc = host_elite(h, h->t + k);
                if (rc) return rc;
            } else if (st == -2) {
                if ((e = launch_chromosome(h->d_desc, h->np, k, n, h->stream)) != hipSuccess)
                    return hip_fail(e, "chromosome-parallel kernel");
            } else if ((e = launch_stage(h->d_desc, blocks, h->R, h->S, st, k, n, h->stream)) !=
                       hipSuccess) {
                return hip_fail(e, "pipeline stage kernel");
            }
            if (h->timing) (void)hipEventRecord(b, h->stream);
        }
    }
    if ((e = launch_finish(h->d_desc, 1, nullptr, n, nullptr, h->stream)) != hipSuccess)
        return hip_fail(e, "finish kernel");
    h->t += n;
    return QIEO_OK;
}

extern "C" int qieo_sync(qieo_inst* h)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (h->onchip_check) {
        h->onchip_check = false;
        uint32_t abort_flag = 0;
        if ((e = copy_on(&abort_flag, h->d.sync + 1, sizeof abort_flag, hipMemcpyDeviceToHost,
                         h->stream)) != hipSuccess)
            return hip_fail(e, "copy(on-chip abort flag)");
        if (abort_flag)
            return set_error(QIEO_EDEVICE, "on-chip loop: a grid barrier wait ran past its bound; "
                                           "the instance's state is undefined");
    }
    if (h->timing) return collect_timing(h);
    return QIEO_OK;
}

extern "C" int qieo_step(qieo_inst* h, int32_t n)
{
    int rc = qieo_step_async(h, n);
    if (rc) return rc;
    return qieo_sync(h);
}

extern "C" int qieo_generations(qieo_inst* h, int64_t* out)
{
    clear_error();
    if (!h || !out) return set_error(QIEO_EINVAL, "NULL argument");
    return read_generations(h->d, h->stream, out);
}

extern "C" int qieo_set_convergence(qieo_inst* h, int32_t window)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (window < 0 || window > kConvRing)
        return set_error(QIEO_EINVAL, "window must be in [0, %d] (got %d)", kConvRing, window);
    if (h->t != 0)
        return set_error(QIEO_ESTATE, "the convergence window is set before the first generation");
    if (window > 0 && h->pipeline != QIEO_PIPELINE_FUSED)
        return set_error(QIEO_ESTATE, "the unfused pipelines do not run the convergence test");
    int rc = write_window(h->d, h->stream, window);
    if (rc == QIEO_OK) h->window = window;
    return rc;
}

extern "C" int qieo_converged(qieo_inst* h, int32_t* converged, int64_t* generation)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    return read_convergence(h->d, h->stream, converged, generation);
}

namespace qieo {

// A small copy ordered on the instance's stream and waited for.  Plain
// hipMemcpy would go through the null stream, a device-wide operation that
// can disturb another thread's graph capture.
hipError_t copy_on(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, n, kind, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Temporary device buffer for reads of an instance's state.
struct TempDev {
    void* p = nullptr;
    explicit TempDev(size_t n)
    {
        if (n == 0) return;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    ~TempDev()
    {
        if (p) (void)hipFree(p);
    }
};

// The best-so-far record and, if bits is not NULL, its alleles unpacked on
// the device into `staging` (device memory of ceil(ng / 32) words; NULL: a
// temporary allocation) and copied to the host.
static int read_best_via(const InstDev& d, int32_t capacity, hipStream_t s, qieo_result* out,
                         uint32_t* bits, size_t n_words, uint32_t* staging)
{
    const size_t need = ((size_t)d.ng + 31) / 32;
    if (bits && n_words < need)
        return set_error(QIEO_EINVAL, "bits buffer has %zu words, needs %zu", n_words, need);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int32_t rec[8];
    if ((e = copy_on(rec, d.best, sizeof rec, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "copy(best)");
    if (!rec[0]) {
        *out = qieo_result{0, 0, 0, 0, -1, -1};
        if (bits) std::memset(bits, 0, need * sizeof(uint32_t));
        return QIEO_OK;
    }
    out->fitness = rec[1];
    out->profit = rec[2];
    out->weight = rec[3];
    out->feasible = rec[3] <= capacity ? 1 : 0;
    out->generation = (int64_t)(((uint64_t)(uint32_t)rec[5] << 32) | (uint32_t)rec[4]);
    out->chromosome = rec[6];
    if (!bits) return QIEO_OK;
    TempDev tmp(staging ? 0 : need * sizeof(uint32_t));
    uint32_t* dst = staging ? staging : (uint32_t*)tmp.p;
    if (!dst) return set_error(QIEO_ENOMEM, "device allocation failed");
    if ((e = launch_bits_unpack(d.best_bits, d.ng, dst, s)) != hipSuccess)
        return hip_fail(e, "bits unpack kernel");
    if ((e = hipMemcpyAsync(bits, dst, need * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(bits)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return QIEO_OK;
}

int read_best(const InstDev& d, int32_t capacity, hipStream_t s, qieo_result* out,
              uint32_t* bits, size_t n_words)
{
    return read_best_via(d, capacity, s, out, bits, n_words, nullptr);
}

int read_generations(const InstDev& d, hipStream_t s, int64_t* t)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = copy_on(t, d.tbase, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "copy(generation counter)");
    return QIEO_OK;
}

int read_convergence(const InstDev& d, hipStream_t s, int32_t* converged, int64_t* generation)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int32_t c[4];
    if ((e = copy_on(c, d.conv, sizeof c, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "copy(convergence)");
    if (converged) *converged = c[3] > 0 ? c[0] : 0;
    if (generation)
        *generation = (c[3] > 0 && c[0]) ? (int64_t)(((uint64_t)(uint32_t)c[2] << 32) | (uint32_t)c[1])
                                        : -1;
    return QIEO_OK;
}

int write_window(const InstDev& d, hipStream_t s, int32_t window)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = copy_on(d.conv + 3, &window, sizeof window, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "copy(window)");
    return QIEO_OK;
}

int export_rows(const InstDev& d, const InstDev* d_desc, hipStream_t s,
                int32_t row0, int32_t n_rows, void* alpha, void* beta, uint8_t* alleles,
                int32_t* fitness, int32_t* profit, int32_t* weight, int32_t* elite, bool f64)
{
    if (row0 < 0 || n_rows < 0 || (int64_t)row0 + n_rows > d.np)
        return set_error(QIEO_EINVAL, "rows [%d, %d) outside [0, %d)", row0, row0 + n_rows, d.np);
    int64_t t = 0;
    int rc0 = read_generations(d, s, &t);
    if (rc0) return rc0;
    hipError_t e;
    if (elite) {
        if (t == 0) {
            *elite = -1;
        } else {
            unsigned long long key = 0;
            if ((e = copy_on(&key, d.ekey + (t - 1) % 3, sizeof key, hipMemcpyDeviceToHost, s)) !=
                hipSuccess)
                return hip_fail(e, "copy(elite)");
            *elite = (int32_t)(~(uint32_t)key);
        }
    }
    if (n_rows == 0) return QIEO_OK;
    const size_t per = (size_t)n_rows * d.ng;
    // device staging only for the outputs asked for
    const size_t amp_bytes = per * (f64 ? sizeof(double) : sizeof(float));
    const size_t row_bytes = (size_t)n_rows * sizeof(int32_t);
    size_t off = 0;
    auto reserve = [&](bool want, size_t n) {
        if (!want) return (size_t)-1;
        const size_t o = off;
        off += (n + 255) / 256 * 256;
        return o;
    };
    const size_t o_a = reserve(alpha != nullptr, amp_bytes);
    const size_t o_b = reserve(beta != nullptr, amp_bytes);
    const size_t o_x = reserve(alleles != nullptr, per);
    const size_t o_f = reserve(fitness != nullptr, row_bytes);
    const size_t o_p = reserve(profit != nullptr, row_bytes);
    const size_t o_w = reserve(weight != nullptr, row_bytes);
    if (off == 0) return QIEO_OK;
    TempDev tmp(off);
    if (!tmp.p) return set_error(QIEO_ENOMEM, "device allocation of %zu bytes failed", off);
    char* base = (char*)tmp.p;
    auto at = [&](size_t o) { return o == (size_t)-1 ? nullptr : base + o; };
    void* da = at(o_a);
    void* db = at(o_b);
    uint8_t* dx = (uint8_t*)at(o_x);
    int32_t* dfit = (int32_t*)at(o_f);
    int32_t* dprof = (int32_t*)at(o_p);
    int32_t* dwt = (int32_t*)at(o_w);
    // the export kernel puts rows on the grid's y dimension (at most 65535):
    // blocks of 32768 rows
    constexpr int32_t kExportRows = 32768;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    for (int32_t r = 0; r < n_rows; r += kExportRows) {
        const int32_t nr = std::min(kExportRows, n_rows - r);
        const size_t o = (size_t)r * d.ng;
        if ((e = launch_export(d_desc, row0 + r, nr, d.ng, da ? (char*)da + o * esz : nullptr,
                               db ? (char*)db + o * esz : nullptr, dx ? dx + o : nullptr,
                               dfit ? dfit + r : nullptr, dprof ? dprof + r : nullptr,
                               dwt ? dwt + r : nullptr, f64, s)) != hipSuccess)
            return hip_fail(e, "export kernel");
    }
    struct { void* dst; const void* src; size_t n; } cp[] = {
        {alpha, da, amp_bytes}, {beta, db, amp_bytes}, {alleles, dx, per},
        {fitness, dfit, row_bytes}, {profit, dprof, row_bytes}, {weight, dwt, row_bytes}};
    int rc = QIEO_OK;
    for (auto& c : cp) {
        if (!c.dst) continue;
        if ((e = hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyDeviceToHost, s)) != hipSuccess) {
            rc = hip_fail(e, "hipMemcpyAsync(export)");
            break;
        }
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess && rc == QIEO_OK)
        rc = hip_fail(e, "hipStreamSynchronize");
    return rc;
}

}  // namespace qieo

extern "C" int qieo_best(qieo_inst* h, qieo_result* out, uint32_t* bits, size_t n_words)
{
    clear_error();
    if (!h || !out) return set_error(QIEO_EINVAL, "NULL argument");
    return read_best(h->d, h->capacity, h->stream, out, bits, n_words);
}

// ---------------------------------------------------------------------------
// qieo_best without allocation.  The unpacked best string goes through a
// file-scope device array (one copy per device, for the process's life).
// Host code never passes `scratch` itself to a kernel or a copy: its name is
// a host-side stand-in; the device address comes from hipGetSymbolAddress,
// taken once per device with that device current.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchWords = QIEO_BEST_NOALLOC_MAX_ITEMS / 32;   // 1 MiB
static_assert(QIEO_BEST_NOALLOC_MAX_ITEMS % 32 == 0, "whole words");
__device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (made current by the caller).
int scratch_on(int dev, uint32_t** out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(QIEO_EDEVICE, "device %d out of range for the static buffer", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_scratch_ptr[dev] = (uint32_t*)p;
    }
    *out = g_scratch_ptr[dev];
    return QIEO_OK;
}
}  // namespace

extern "C" int qieo_best_noalloc(qieo_inst* h, qieo_result* out, uint32_t* bits, size_t n_words)
{
    clear_error();
    if (!h || !out) return set_error(QIEO_EINVAL, "NULL argument");
    if (bits && (size_t)h->ng > (size_t)QIEO_BEST_NOALLOC_MAX_ITEMS)
        return set_error(QIEO_EINVAL, "%d items exceed the static staging of %d items", h->ng,
                         QIEO_BEST_NOALLOC_MAX_ITEMS);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != h->device && (e = hipSetDevice(h->device)) != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    uint32_t* staging = nullptr;
    int rc = bits ? scratch_on(h->device, &staging) : QIEO_OK;
    if (rc == QIEO_OK) rc = read_best_via(h->d, h->capacity, h->stream, out, bits, n_words, staging);
    if (cur != h->device) (void)hipSetDevice(cur);
    return rc;
}

extern "C" int qieo_export_rows(qieo_inst* h, int32_t row0, int32_t n_rows, float* alpha,
                                float* beta, uint8_t* alleles, int32_t* fitness,
                                int32_t* profit, int32_t* weight, int32_t* elite)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (h->f64 && (alpha || beta))
        return set_error(QIEO_EINVAL, "binary64 instance: use qieo_export_rows_f64");
    return export_rows(h->d, h->d_desc, h->stream, row0, n_rows, alpha, beta, alleles,
                       fitness, profit, weight, elite, false);
}

extern "C" int qieo_export_rows_f64(qieo_inst* h, int32_t row0, int32_t n_rows, double* alpha,
                                    double* beta, uint8_t* alleles, int32_t* fitness,
                                    int32_t* profit, int32_t* weight, int32_t* elite)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (!h->f64 && (alpha || beta))
        return set_error(QIEO_EINVAL, "binary32 instance: use qieo_export_rows");
    return export_rows(h->d, h->d_desc, h->stream, row0, n_rows, alpha, beta, alleles,
                       fitness, profit, weight, elite, true);
}

extern "C" void qieo_destroy(qieo_inst* h) { inst_release(h); }

extern "C" int qieo_set_tile(qieo_inst* h, int32_t rows_per_block, int32_t waves_per_block)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (rows_per_block != 0 && rows_per_block != 1 && rows_per_block != 2 && rows_per_block != 4)
        return set_error(QIEO_EINVAL, "rows_per_block must be 1, 2 or 4 (got %d)",
                         rows_per_block);
    if (waves_per_block < 0 || waves_per_block > 16)
        return set_error(QIEO_EINVAL, "waves_per_block must be in [1, 16] (got %d)",
                         waves_per_block);
    int R, S, F;
    default_shape(h, &R, &S, &F);
    h->R = rows_per_block ? rows_per_block : R;
    h->S = waves_per_block ? waves_per_block : S;
    return QIEO_OK;
}

extern "C" int qieo_set_kernel_flags(qieo_inst* h, int32_t flags)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (flags < 0 || flags > kFlagAll)
        return set_error(QIEO_EINVAL, "flags must be in [0, %d] (got %d)", kFlagAll, flags);
    h->flags = flags;
    return QIEO_OK;
}

extern "C" int qieo_get_kernel_flags(qieo_inst* h, int32_t* flags)
{
    clear_error();
    if (!h || !flags) return set_error(QIEO_EINVAL, "NULL argument");
    *flags = h->flags;
    return QIEO_OK;
}

extern "C" int qieo_get_tile(qieo_inst* h, int32_t* rows_per_block, int32_t* waves_per_block)
{
    clear_error();
    if (!h || !rows_per_block || !waves_per_block) return set_error(QIEO_EINVAL, "NULL argument");
    *rows_per_block = h->R;
    *waves_per_block = h->S;
    return QIEO_OK;
}

extern "C" int qieo_set_barrier_timeout(qieo_inst* h, int64_t microseconds)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (microseconds < 0 || microseconds > 3600LL * 1000000)
        return set_error(QIEO_EINVAL, "timeout must be in [0, 3600 s] (got %lld us)",
                         (long long)microseconds);
    h->barrier_us = microseconds;
    return QIEO_OK;
}

extern "C" int qieo_get_call_path(qieo_inst* h, int32_t* path)
{
    clear_error();
    if (!h || !path) return set_error(QIEO_EINVAL, "NULL argument");
    *path = h->last_path;
    return QIEO_OK;
}

extern "C" int qieo_set_timing(qieo_inst* h, int enabled)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    h->timing = enabled != 0;
    return QIEO_OK;
}

extern "C" int qieo_kernel_time(qieo_inst* h, int64_t* launches, double* total_ms, int reset)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    int rc = collect_timing(h);
    if (rc) return rc;
    if (launches) *launches = h->launches[0];
    if (total_ms) *total_ms = h->total_ms[0];
    if (reset) {
        h->launches[0] = 0;
        h->total_ms[0] = 0.0;
    }
    return QIEO_OK;
}

extern "C" int qieo_stage_time(qieo_inst* h, int64_t* launches, double* total_ms, int reset)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    int rc = collect_timing(h);
    if (rc) return rc;
    for (int i = 0; i < kStages; ++i) {
        if (launches) launches[i] = h->launches[i];
        if (total_ms) total_ms[i] = h->total_ms[i];
        if (reset) {
            h->launches[i] = 0;
            h->total_ms[i] = 0.0;
        }
    }
    return QIEO_OK;
}

extern "C" int qieo_set_graph(qieo_inst* h, int32_t enabled)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    h->use_graph = enabled != 0;
    return QIEO_OK;
}

extern "C" int qieo_set_persistent(qieo_inst* h, int32_t mode)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (mode < 0 || mode > 3)
        return set_error(QIEO_EINVAL, "mode must be 0, 1, 2 or 3 (got %d)", mode);
    if (h->f64 && mode != 0)
        return set_error(QIEO_ESTATE, "binary64 instances use per-generation launches");
    h->persistent = mode;
    return QIEO_OK;
}

extern "C" int qieo_set_pipeline(qieo_inst* h, int32_t pipeline)
{
    clear_error();
    if (!h) return set_error(QIEO_EINVAL, "handle is NULL");
    if (pipeline < QIEO_PIPELINE_FUSED || pipeline > QIEO_PIPELINE_CHROMOSOME)
        return set_error(QIEO_EINVAL, "unknown pipeline %d", pipeline);
    if (pipeline != QIEO_PIPELINE_FUSED && h->window > 0)
        return set_error(QIEO_ESTATE, "the unfused pipelines do not run the convergence test");
    if (pipeline != QIEO_PIPELINE_FUSED && h->f64)
        return set_error(QIEO_ESTATE, "binary64 instances run the fused pipeline only");
    if (pipeline == QIEO_PIPELINE_UNFUSED_HOST_DE && !h->h_fit) {
        hipError_t e;
        if ((e = hipHostMalloc((void**)&h->h_fit, (size_t)h->np * sizeof(int32_t),
                               hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "hipHostMalloc");
        if ((e = hipHostMalloc((void**)&h->h_key, sizeof(unsigned long long),
                               hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "hipHostMalloc");
    }
    h->pipeline = pipeline;
    return QIEO_OK;
}

extern "C" const char* qieo_strerror(int code)
{
    switch (code) {
    case QIEO_OK: return "success";
    case QIEO_EINVAL: return "invalid argument";
    case QIEO_EOVERFLOW: return "sum of profits or weights exceeds INT32_MAX";
    case QIEO_ENOMEM: return "out of memory";
    case QIEO_EDEVICE: return "device or HIP runtime error";
    case QIEO_EAGAIN: return "not ready";
    case QIEO_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

extern "C" const char* qieo_last_error(void) { return last_error(); }

extern "C" const char* qieo_version(void) { return "libqieo 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// Checkpoint and resume.  A snapshot is a fixed header followed by the whole
// device arena: amplitude planes (the last generation's rotation still
// pending), allele words, item tables, fitness slots, elite keys, best record
// and bits, generation counter and convergence state.  Loading it into a
// handle of the same problem restores every value the kernels read, so the
// trajectory continues bit for bit.
// ---------------------------------------------------------------------------
static SnapshotId snapshot_id(const qieo_inst* h)
{
    return SnapshotId{h->f64 ? 8u : 4u, h->ng, h->np, h->capacity, h->seed, h->items_hash};
}

extern "C" int qieo_state_size(qieo_inst* h, size_t* bytes)
{
    clear_error();
    if (!h || !bytes) return set_error(QIEO_EINVAL, "NULL argument");
    *bytes = sizeof(StateHeader) + h->L.total;
    return QIEO_OK;
}

extern "C" int qieo_export_state(qieo_inst* h, void* buf, size_t bytes)
{
    clear_error();
    if (!h || !buf) return set_error(QIEO_EINVAL, "NULL argument");
    const size_t need = sizeof(StateHeader) + h->L.total;
    if (bytes < need)
        return set_error(QIEO_EINVAL, "state buffer has %zu bytes, needs %zu", bytes, need);
    int64_t t = 0;
    int rc = read_generations(h->d, h->stream, &t);
    if (rc) return rc;
    const StateHeader hd = make_state_header(snapshot_id(h), t, h->L.total);
    std::memcpy(buf, &hd, sizeof hd);
    hipError_t e = copy_on((char*)buf + sizeof hd, h->arena, h->L.total, hipMemcpyDeviceToHost,
                           h->stream);
    if (e != hipSuccess) return hip_fail(e, "copy(state)");
    return QIEO_OK;
}

extern "C" int qieo_import_state(qieo_inst* h, const void* buf, size_t bytes)
{
    clear_error();
    if (!h || !buf) return set_error(QIEO_EINVAL, "NULL argument");
    int64_t tb = 0;
    int32_t window = 0;
    int rc = check_snapshot(buf, bytes, snapshot_id(h), h->L, &tb, &window);
    if (rc) return rc;
    const char* body = (const char*)buf + sizeof(StateHeader);
    if (window > 0 && h->pipeline != QIEO_PIPELINE_FUSED)
        return set_error(QIEO_ESTATE, "snapshot has a convergence window: select the fused "
                                      "pipeline first");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = copy_on(h->arena, body, h->L.total, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return hip_fail(e, "copy(state)");
    h->t = tb;
    h->window = window;
    return QIEO_OK;
}
