// Multi-instance engine and the batch C ABI.
//
// A batch keeps every population resident in one device pool and advances
// all of them with the same generation launches: the tile table of a launch
// lists (instance, first row) pairs from every instance of one shape class,
// so a generation of 512 small instances costs a handful of launches instead
// of 512.  The launches of a whole call (n generations x classes, plus the
// finishing step) are captured once into a HIP graph and replayed.
#include "qieo_multi.hpp"
#include "qieo_onchip.hpp"

#include <algorithm>
#include <functional>
#include <cstring>
#include <new>

#include "../../include/qieo.h"

namespace qieo {

// ---------------------------------------------------------------------------
// DevicePool
// ---------------------------------------------------------------------------
static size_t round256(size_t x) { return (x + 255) / 256 * 256; }

DevicePool::~DevicePool()
{
    mem_.release(base_);
}

int DevicePool::init(size_t bytes, const qieo_dev_ctx* ctx)
{
    bytes = round256(std::max<size_t>(bytes, 256));
    mem_.set(ctx);
    base_ = (char*)mem_.alloc(bytes);
    if (!base_) return set_error(QIEO_ENOMEM, "device pool of %zu bytes could not be allocated", bytes);
    book_.reset(bytes);
    return QIEO_OK;
}

char* DevicePool::alloc(size_t bytes)
{
    const size_t off = book_.alloc(bytes);
    return off == OffsetAllocator::npos ? nullptr : base_ + off;
}

void DevicePool::release(char* p)
{
    if (p) (void)book_.release((size_t)(p - base_));
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
Engine::~Engine()
{
    if (stream_) (void)hipStreamSynchronize(stream_);
    if (side_) (void)hipStreamSynchronize(side_);
    for (hipStream_t cs : cstreams_) (void)hipStreamSynchronize(cs);
    invalidate_graph();
    mem_.release(d_pids_);
    if (fork_) (void)hipEventDestroy(fork_);
    if (join_) (void)hipEventDestroy(join_);
    if (side_) (void)hipStreamDestroy(side_);
    for (hipEvent_t ev : cjoin_) (void)hipEventDestroy(ev);
    for (hipStream_t cs : cstreams_) (void)hipStreamDestroy(cs);
    for (auto& c : classes_) {
        mem_.release(c.d_tiles);
        mem_.release(c.d_fe_tiles);
    }
    for (auto& o : onchip_) mem_.release(o.d_tiles);
    mem_.release(d_abort_);
    mem_.release(d_desc_);
    mem_.release(d_gens_);
    mem_.release(d_status_);
    if (h_gens_) (void)hipHostFree(h_gens_);
}

void Engine::invalidate_graph()
{
    if (graph_) (void)hipGraphExecDestroy(graph_);
    graph_ = nullptr;
    graph_n_ = -1;
}

int Engine::add(DevicePool& pool, const qieo_item* items, int32_t n_items, int32_t capacity,
                int32_t n_pop, uint64_t seed, uint64_t id, int32_t window)
{
    int rc = validate_problem(items, n_items, capacity, n_pop);
    if (rc) return rc;
    Member m;
    arena_layout(n_items, n_pop, &m.L);
    m.arena = pool.alloc(m.L.total);
    if (!m.arena)
        return set_error(QIEO_ENOMEM, "no room for %zu bytes in the device pool (%zu of %zu used)",
                         m.L.total, pool.used(), pool.capacity());
    m.d = bind_arena(m.arena, m.L, n_items, n_pop, capacity, seed);
    m.ng = n_items;
    m.np = n_pop;
    m.packed = items_packable(items, n_items);
    m.capacity = capacity;
    m.seed = seed;
    m.id = id;
    if ((rc = upload_and_init(m.d, items, stream_, m.L, m.arena, staging_))) {
        pool.release(m.arena);
        return rc;
    }
    // the pageable staging buffer is reused by the next add
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) {
        pool.release(m.arena);
        return hip_fail(e, "hipStreamSynchronize");
    }
    if (window > 0 && (rc = write_window(m.d, stream_, window))) {
        pool.release(m.arena);
        return rc;
    }
    m.window = window;
    members_.push_back(m);
    dirty_ = true;
    return QIEO_OK;
}

void Engine::remove_at(size_t idx, DevicePool& pool)
{
    if (idx >= members_.size()) return;
    pool.release(members_[idx].arena);
    members_.erase(members_.begin() + idx);
    dirty_ = true;
}

void Engine::force_shape(int R, int S, int flags)
{
    force_R_ = R;
    force_S_ = S;
    force_flags_ = flags;
    dirty_ = true;
}

int Engine::rebuild()
{
    invalidate_graph();
    prev_n_ = -1;
    // the tables below are freed and replaced: no queued launch may still
    // read them (a caller's allocator may hand their memory out again at once)
    {
        const hipError_t se = hipStreamSynchronize(stream_);
        if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    }
    // the abort words of a call not yet synchronised are read before they go
    {
        const int rc0 = check_onchip_abort();
        if (rc0) return rc0;
    }
    for (auto& c : classes_) {
        mem_.release(c.d_tiles);
        mem_.release(c.d_fe_tiles);
    }
    classes_.clear();
    for (auto& o : onchip_) mem_.release(o.d_tiles);
    onchip_.clear();
    mem_.release(d_abort_);
    d_abort_ = nullptr;
    const size_t n = members_.size();
    hipError_t e;
    // copies from the local host vectors below may still be in flight when a
    // later step fails: drain the stream before they go out of scope
    auto rebuild_fail = [&](hipError_t err, const char* what) {
        (void)hipStreamSynchronize(stream_);
        (void)hipGetLastError();
        return hip_fail(err, what);
    };
    auto rebuild_nomem = [&](const char* what) {
        (void)hipStreamSynchronize(stream_);
        return set_error(QIEO_ENOMEM, "device allocation of the %s failed", what);
    };
    if (n > desc_cap_) {
        // the tables grow to twice their size (or n); they are unusable until
        // every allocation below has succeeded
        const size_t cap = std::max<size_t>(n, 2 * desc_cap_);
        mem_.release(d_desc_);
        mem_.release(d_gens_);
        mem_.release(d_status_);
        if (h_gens_) (void)hipHostFree(h_gens_);
        d_desc_ = nullptr;
        d_gens_ = nullptr;
        d_status_ = nullptr;
        h_gens_ = nullptr;
        desc_cap_ = gens_cap_ = 0;
        if (!(d_desc_ = (InstDev*)mem_.alloc(cap * sizeof(InstDev))))
            return set_error(QIEO_ENOMEM, "device allocation of the descriptors failed");
        if (!(d_gens_ = (int32_t*)mem_.alloc(cap * sizeof(int32_t))))
            return set_error(QIEO_ENOMEM, "device allocation of the generation counts failed");
        if (!(d_status_ = (int64_t*)mem_.alloc(2 * cap * sizeof(int64_t))))
            return set_error(QIEO_ENOMEM, "device allocation of the status words failed");
        if ((e = hipHostMalloc((void**)&h_gens_, cap * sizeof(int32_t), hipHostMallocDefault)) !=
            hipSuccess)
            return hip_fail(e, "hipHostMalloc");
        desc_cap_ = gens_cap_ = cap;
    }
    if (n == 0) {
        dirty_ = false;
        return QIEO_OK;
    }
    std::vector<InstDev> desc(n);
    for (size_t i = 0; i < n; ++i) desc[i] = members_[i].d;
    if ((e = hipMemcpyAsync(d_desc_, desc.data(), n * sizeof(InstDev), hipMemcpyHostToDevice,
                            stream_)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(descriptors)");

    // resident set, shape classes and tile tables (host planning)
    std::vector<MemberShape> shapes(n);
    for (size_t i = 0; i < n; ++i) {
        const Member& m = members_[i];
        shapes[i].np = m.np;
        shapes[i].pitch = m.L.pitch;
        shapes[i].nchunk = m.L.nchunk;
        shapes[i].part_nseg = m.L.part_nseg;
        shapes[i].addr = (uint64_t)(uintptr_t)m.arena;
        shapes[i].conv = m.window > 0;
        shapes[i].packed = m.packed;
    }
    PlanOptions opt;
    opt.use_persistent = use_persistent_;
    opt.lds_limit = use_persistent_ ? resident_lds_limit() : 0;
    opt.use_segments = use_segments_;
    opt.merge_segments = merge_segments_;
    opt.force_R = force_R_;
    opt.force_S = force_S_;
    opt.force_flags = force_flags_;
    opt.tuned = use_tuned_ ? tuned_class : nullptr;
    set_onchip_options(&opt);
    BatchPlan plan;
    int rc = plan_batch(shapes, opt, &plan);
    if (rc) {
        (void)hipStreamSynchronize(stream_);
        return rc;
    }
    pids_ = std::move(plan.resident);
    pids_lds_ = plan.resident_lds;
    mem_.release(d_pids_);
    d_pids_ = nullptr;
    if (!pids_.empty()) {
        if (!(d_pids_ = (uint32_t*)mem_.alloc(pids_.size() * sizeof(uint32_t))))
            return rebuild_nomem("persistent ids");
        if ((e = hipMemcpyAsync(d_pids_, pids_.data(), pids_.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, stream_)) != hipSuccess)
            return rebuild_fail(e, "hipMemcpyAsync(persistent ids)");
        if (!side_) {
            if ((e = hipStreamCreateWithFlags(&side_, hipStreamNonBlocking)) != hipSuccess)
                return rebuild_fail(e, "hipStreamCreate");
            if ((e = hipEventCreateWithFlags(&join_, hipEventDisableTiming)) != hipSuccess)
                return rebuild_fail(e, "hipEventCreate");
        }
    }
    if (!fork_ && (e = hipEventCreateWithFlags(&fork_, hipEventDisableTiming)) != hipSuccess)
        return rebuild_fail(e, "hipEventCreate");
    if (!plan.onchip.empty()) {
        if (!(d_abort_ = (uint32_t*)mem_.alloc(plan.onchip.size() * sizeof(uint32_t))))
            return rebuild_nomem("on-chip abort words");
        for (OnchipLaunch& L : plan.onchip) {
            // owned by onchip_ from here on (freed at the next rebuild)
            onchip_.push_back(OnchipRun{L.K, L.conv, L.packed, L.lds, (int)L.tiles.size(), nullptr});
            OnchipRun& o = onchip_.back();
            if (!(o.d_tiles = (OnchipTile*)mem_.alloc(L.tiles.size() * sizeof(OnchipTile))))
                return rebuild_nomem("on-chip tiles");
            if ((e = hipMemcpyAsync(o.d_tiles, L.tiles.data(), L.tiles.size() * sizeof(OnchipTile),
                                    hipMemcpyHostToDevice, stream_)) != hipSuccess)
                return rebuild_fail(e, "hipMemcpyAsync(on-chip tiles)");
        }
    }
    for (ClassPlan& cp : plan.classes) {
        ShapeClass sc;
        sc.cls = cp.cls;
        sc.R = cp.R;
        sc.S = cp.S;
        sc.flags = cp.flags;
        sc.tuned = cp.tuned;
        sc.tiles = std::move(cp.tiles);
        sc.fe_tiles = std::move(cp.fe_tiles);
        // owned by classes_ from here on, so an early return frees the tables
        // at the next rebuild or in the destructor
        classes_.push_back(std::move(sc));
        ShapeClass& cc = classes_.back();
        if (!(cc.d_tiles = (Tile*)mem_.alloc(cc.tiles.size() * sizeof(Tile))))
            return rebuild_nomem("tiles");
        if ((e = hipMemcpyAsync(cc.d_tiles, cc.tiles.data(), cc.tiles.size() * sizeof(Tile),
                                hipMemcpyHostToDevice, stream_)) != hipSuccess)
            return rebuild_fail(e, "hipMemcpyAsync(tiles)");
        if (!cc.fe_tiles.empty()) {
            if (!(cc.d_fe_tiles = (Tile*)mem_.alloc(cc.fe_tiles.size() * sizeof(Tile))))
                return rebuild_nomem("tiles");
            if ((e = hipMemcpyAsync(cc.d_fe_tiles, cc.fe_tiles.data(),
                                    cc.fe_tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                                    stream_)) != hipSuccess)
                return rebuild_fail(e, "hipMemcpyAsync(tiles)");
        }
    }
    while (cstreams_.size() + 1 < classes_.size()) {
        hipStream_t cs = nullptr;
        hipEvent_t ev = nullptr;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
            return rebuild_fail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return rebuild_fail(e, "hipEventCreate");
        }
        cstreams_.push_back(cs);
        cjoin_.push_back(ev);
    }
    // host vectors above are pageable and local: wait for their copies
    if ((e = hipStreamSynchronize(stream_)) != hipSuccess)
        return rebuild_fail(e, "hipStreamSynchronize");
    dirty_ = false;
    return QIEO_OK;
}

// Members of different shape classes (and the LDS-resident members) share
// nothing, so each class advances through all of its generations on a stream
// of its own, forked from the main stream and joined back before the
// finishing launch: a small class's launches overlap the large classes'
// instead of queueing behind them every generation.
int Engine::enqueue(int nmax)
{
    hipError_t e;
    // the batched on-chip launches first, alone on the device: a cooperative
    // launch holds its workgroups' CUs for the whole call, so nothing of this
    // call runs beside it
    if (!onchip_.empty()) {
        const int64_t ticks = onchip_spin_ticks(device_of_stream(), barrier_us_);
        // set first: launches enqueued before a failing one still get their
        // abort words read at the next sync
        onchip_check_ = true;
        for (size_t j = 0; j < onchip_.size(); ++j) {
            const OnchipRun& o = onchip_[j];
            if ((e = launch_onchip_multi(d_desc_, o.d_tiles, o.n_tiles, o.K, o.conv, o.packed, o.lds,
                                         d_gens_, 0, d_abort_ + j, ticks, stream_)) != hipSuccess)
                return hip_fail(e, "batched on-chip kernel");
        }
    }
    const size_t nc = classes_.size();
    const bool forked = !pids_.empty() || nc > 1;
    if (forked && (e = hipEventRecord(fork_, stream_)) != hipSuccess) return hip_fail(e, "fork");
    if (!pids_.empty()) {
        if ((e = hipStreamWaitEvent(side_, fork_, 0)) != hipSuccess) return hip_fail(e, "fork");
        if ((e = launch_resident(d_desc_, d_pids_, (int)pids_.size(), 8, pids_lds_, d_gens_, 0,
                                 side_)) != hipSuccess)
            return hip_fail(e, "resident kernel");
        if ((e = hipEventRecord(join_, side_)) != hipSuccess) return hip_fail(e, "join");
    }
    // Class after class, smallest rows first: the small classes'
    // launch-bound generations run while the host is still issuing the
    // long-row class's.  Issued generation by generation across the class
    // streams instead (long rows first in each round), the long-row stream
    // starts at once but shares the chip with the small kernels all along:
    // 0.333 s against 0.330 s per call on the 512-instance batch.
    for (size_t ci = 0; ci < nc; ++ci) {
        const ShapeClass& c = classes_[ci];
        hipStream_t cs = ci == 0 ? stream_ : cstreams_[ci - 1];
        if (ci > 0 && (e = hipStreamWaitEvent(cs, fork_, 0)) != hipSuccess)
            return hip_fail(e, "fork");
        for (int k = 0; k < nmax; ++k) {
            e = (c.flags & kFlagSegments)
                    ? launch_segments_tiled(d_desc_, c.d_tiles, (int)c.tiles.size(),
                                            c.d_fe_tiles, (int)c.fe_tiles.size(), c.flags, k,
                                            d_gens_, cs)
                    : launch_generation(d_desc_, c.d_tiles, (int)c.tiles.size(), c.R, c.S,
                                        c.flags, k, d_gens_, 0, cs);
            if (e != hipSuccess) return hip_fail(e, "generation kernel");
        }
        if (ci > 0 && (e = hipEventRecord(cjoin_[ci - 1], cs)) != hipSuccess)
            return hip_fail(e, "join");
    }
    for (size_t ci = 1; ci < nc; ++ci)
        if ((e = hipStreamWaitEvent(stream_, cjoin_[ci - 1], 0)) != hipSuccess)
            return hip_fail(e, "join");
    if (!pids_.empty() && (e = hipStreamWaitEvent(stream_, join_, 0)) != hipSuccess)
        return hip_fail(e, "join");
    if ((e = launch_finish(d_desc_, (int)members_.size(), d_gens_, 0, d_status_, stream_)) !=
        hipSuccess)
        return hip_fail(e, "finish kernel");
    return QIEO_OK;
}

// Relaxed mode: the captured sequence holds launches, event records and
// waits only.  Returns false, with no graph and the error state clear, if the
// capture does not complete (another thread's device-wide call can
// invalidate a capture in progress); the caller then enqueues directly.
bool Engine::capture(int nmax)
{
    invalidate_graph();
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(stream_, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        clear_error();
        return false;
    }
    const int rc = enqueue(nmax);
    const hipError_t e = hipStreamEndCapture(stream_, &g);
    hipGraphExec_t x = nullptr;
    if (rc == QIEO_OK && e == hipSuccess && g &&
        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
        graph_ = x;
        graph_n_ = nmax;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    clear_error();
    return graph_ != nullptr;
}

int Engine::run(const int32_t* gens)
{
    int rc;
    if (dirty_ && (rc = rebuild())) return rc;
    const size_t n = members_.size();
    if (n == 0) return QIEO_OK;
    int nmax = 0;
    for (size_t i = 0; i < n; ++i) {
        if (gens[i] < 0) return set_error(QIEO_EINVAL, "negative generation count for instance %zu", i);
        if (members_[i].t + gens[i] > (int64_t)INT32_MAX)
            return set_error(QIEO_EINVAL, "generation index of instance %zu would exceed 2^31-1", i);
        nmax = std::max(nmax, gens[i]);
    }
    if (nmax == 0) return QIEO_OK;
    // the pinned counts may still feed the previous call's copy
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::memcpy(h_gens_, gens, n * sizeof(int32_t));
    if ((e = hipMemcpyAsync(d_gens_, h_gens_, n * sizeof(int32_t), hipMemcpyHostToDevice,
                            stream_)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(generation counts)");
    // a call is captured once it repeats (same longest count, same members):
    // capturing a one-off call costs more than launching it
    const bool repeat = prev_n_ == nmax;
    prev_n_ = nmax;
    bool done = false;
    // a cooperative launch is not captured: a batch with on-chip launches
    // enqueues its calls directly
    if (use_graph_ && onchip_.empty() && (graph_n_ == nmax || (repeat && capture(nmax)))) {
        if ((e = hipGraphLaunch(graph_, stream_)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        done = true;
    }
    if (!done) {
        // a side stream left in a lost capture cannot be used
        std::vector<hipStream_t> forks(cstreams_);
        if (side_) forks.push_back(side_);
        for (hipStream_t fs : forks) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(fs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                return set_error(QIEO_EDEVICE, "side stream left capturing by a lost graph capture");
        }
        if ((rc = enqueue(nmax))) return rc;
    }
    for (size_t i = 0; i < n; ++i) members_[i].t += gens[i];
    return QIEO_OK;
}

int Engine::sync()
{
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return check_onchip_abort();
}

// After the stream has drained: fails if a batched on-chip launch queued
// since the last check gave up on a barrier wait.
int Engine::check_onchip_abort()
{
    if (!onchip_check_) return QIEO_OK;
    onchip_check_ = false;
    std::vector<uint32_t> flags(onchip_.size(), 0u);
    hipError_t e;
    if (!flags.empty() &&
        (e = copy_on(flags.data(), d_abort_, flags.size() * sizeof(uint32_t),
                     hipMemcpyDeviceToHost, stream_)) != hipSuccess)
        return hip_fail(e, "copy(on-chip abort words)");
    for (uint32_t f : flags)
        if (f)
            return set_error(QIEO_EDEVICE, "batched on-chip loop: a barrier wait ran past its "
                                           "bound; the state of its members is undefined");
    return QIEO_OK;
}

// Device the engine's stream belongs to.
int Engine::device_of_stream() const
{
    int dev = 0;
    if (hipStreamGetDevice(stream_, &dev) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGetDevice(&dev);
    }
    return dev;
}

// Rows of all members and the longest row in chunks: the tuning database's
// bucket for a batch's on-chip variant subset.
void Engine::batch_signature(int64_t* rows, int32_t* max_nchunk) const
{
    *rows = 0;
    *max_nchunk = 0;
    for (const Member& m : members_) {
        *rows += m.np;
        *max_nchunk = std::max(*max_nchunk, m.L.nchunk);
    }
}

void Engine::set_onchip_options(PlanOptions* opt) const
{
    if (!use_onchip_) return;
    size_t lim = 0;
    int ncu = 0;
    onchip_limits(&lim, &ncu);
    // the subset tuned on this batch, else one tuned on a batch of the same
    // bucket, else every usable variant
    unsigned mask = onchip_mask_;
    int R = 0, S = 0, F = 0;
    int64_t rows = 0;
    int32_t maxc = 0;
    batch_signature(&rows, &maxc);
    if (!mask && use_tuned_ && tuned_class(-1, rows, maxc, &R, &S, &F)) mask = (unsigned)F;
    opt->onchip_blocks = ncu;
    opt->onchip_lds_limit = lim;
    opt->onchip_variants = ncu > 0 ? onchip_multi_variants() & (mask ? mask : ~0u) : 0u;
}

int Engine::refresh_status()
{
    const size_t n = members_.size();
    if (n == 0 || !d_status_) return QIEO_OK;
    std::vector<int64_t> st(2 * n);
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int rc = check_onchip_abort();
    if (rc) return rc;
    if ((e = copy_on(st.data(), d_status_, st.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                     stream_)) != hipSuccess)
        return hip_fail(e, "copy(status)");
    for (size_t i = 0; i < n; ++i) {
        members_[i].t = st[2 * i];
        members_[i].converged = st[2 * i + 1] != 0;
    }
    return QIEO_OK;
}

// The batched on-chip launches' variant subset, timed on the batch itself:
// every subset of the usable variants that holds the largest one (so every
// member the current plan places stays placeable), planned for the members
// the current plan places, each run for gens generations of all its
// launches from the saved state, twice in opposite orders, the faster time
// counting.  The fastest subset is kept for this batch (onchip_mask_) and
// reported as an entry with shape_class -1.
int Engine::tune_onchip(int gens, const std::vector<MemberShape>& shapes, const PlanOptions& opt,
                        const BatchPlan& plan,
                        const std::function<hipError_t(const std::vector<uint32_t>&)>& restore,
                        std::vector<void*>& temps, hipEvent_t e0, hipEvent_t e1,
                        std::vector<qieo_class_tune>* out)
{
    std::vector<uint32_t> ids;
    {
        std::vector<bool> seen(members_.size(), false);
        for (const OnchipLaunch& L : plan.onchip)
            for (const OnchipTile& t : L.tiles)
                if (!seen[t.inst]) {
                    seen[t.inst] = true;
                    ids.push_back(t.inst);
                }
        std::sort(ids.begin(), ids.end());
    }
    std::vector<size_t> cand_ids(ids.begin(), ids.end());
    const unsigned usable = onchip_multi_variants();
    int top = -1;
    for (int v = 0; v < kOnchipVariants; ++v)
        if (usable & (1u << v)) top = v;
    if (top < 0) return QIEO_OK;
    struct Cand {
        unsigned mask;
        std::vector<OnchipLaunch> launches;
        std::vector<OnchipTile*> d_tiles;
        double ms;
    };
    std::vector<Cand> cand;
    size_t max_launches = 0;
    int64_t rows = 0;
    int32_t max_chunks = 0;
    for (uint32_t i : ids) {
        rows += members_[i].np;
        max_chunks = std::max(max_chunks, members_[i].L.nchunk);
    }
    for (unsigned m = 1; m < (1u << kOnchipVariants); ++m) {
        if ((m & usable) != m || !(m & (1u << top))) continue;
        PlanOptions o = opt;
        o.onchip_variants = m;
        Cand c{m, {}, {}, 1e300};
        std::vector<size_t> rest;
        plan_onchip(shapes, cand_ids, o, &c.launches, &rest);
        if (!rest.empty() || c.launches.empty()) continue;
        for (const OnchipLaunch& L : c.launches) {
            OnchipTile* d = (OnchipTile*)mem_.alloc(L.tiles.size() * sizeof(OnchipTile));
            if (!d) return set_error(QIEO_ENOMEM, "device allocation of tuning tiles failed");
            temps.push_back(d);
            const hipError_t ee = hipMemcpyAsync(d, L.tiles.data(), L.tiles.size() * sizeof(OnchipTile),
                                                 hipMemcpyHostToDevice, stream_);
            if (ee != hipSuccess) return hip_fail(ee, "hipMemcpyAsync(tiles)");
            c.d_tiles.push_back(d);
        }
        max_launches = std::max(max_launches, c.launches.size());
        cand.push_back(std::move(c));
    }
    if (cand.empty()) return QIEO_OK;
    uint32_t* d_abort = (uint32_t*)mem_.alloc(max_launches * sizeof(uint32_t));
    if (!d_abort) return set_error(QIEO_ENOMEM, "device allocation of tuning abort words failed");
    temps.push_back(d_abort);
    // the tile tables above are local host vectors: their copies complete here
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int64_t ticks = onchip_spin_ticks(device_of_stream(), barrier_us_);
    auto time_one = [&](Cand& c) {
        hipError_t ee = restore(ids);
        if (ee == hipSuccess) ee = hipEventRecord(e0, stream_);
        for (size_t j = 0; j < c.launches.size() && ee == hipSuccess; ++j)
            ee = launch_onchip_multi(d_desc_, c.d_tiles[j], (int)c.launches[j].tiles.size(),
                                     c.launches[j].K, c.launches[j].conv, c.launches[j].packed,
                                     c.launches[j].lds, d_gens_, 0, d_abort + j, ticks, stream_);
        if (ee == hipSuccess) ee = hipEventRecord(e1, stream_);
        if (ee == hipSuccess) ee = hipEventSynchronize(e1);
        float ms = 0.f;
        if (ee == hipSuccess) ee = hipEventElapsedTime(&ms, e0, e1);
        if (ee != hipSuccess) return hip_fail(ee, "tuning launch");
        std::vector<uint32_t> flags(c.launches.size(), 0u);
        if ((ee = copy_on(flags.data(), d_abort, flags.size() * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, stream_)) != hipSuccess)
            return hip_fail(ee, "copy(on-chip abort words)");
        for (uint32_t f : flags)
            if (f)
                return set_error(QIEO_EDEVICE, "batched on-chip loop: a barrier wait ran past "
                                               "its bound while tuning");
        c.ms = std::min(c.ms, (double)ms / gens);
        return QIEO_OK;
    };
    int rc;
    for (int pass = 0; pass < 2; ++pass)
        for (size_t j = 0; j < cand.size(); ++j)
            if ((rc = time_one(cand[pass == 0 ? j : cand.size() - 1 - j]))) return rc;
    const unsigned dflt_mask = opt.onchip_variants;
    const Cand* best = &cand[0];
    const Cand* dflt = nullptr;
    for (const Cand& c : cand) {
        if (c.ms < best->ms) best = &c;
        if (c.mask == dflt_mask) dflt = &c;
    }
    onchip_mask_ = best->mask;
    {
        int64_t all_rows = 0;
        int32_t all_max = 0;
        batch_signature(&all_rows, &all_max);
        record_class(-1, all_rows, all_max, (int)best->launches.size(), kOnchipWaves,
                     (int)best->mask, best->ms);
    }
    qieo_class_tune r{};
    r.shape_class = -1;
    r.rows = (int32_t)std::min<int64_t>(rows, INT32_MAX);
    r.max_chunks = max_chunks;
    r.rows_per_block = (int32_t)best->launches.size();
    r.waves_per_block = kOnchipWaves;
    r.flags = (int32_t)best->mask;
    r.default_rows_per_block = (int32_t)plan.onchip.size();
    r.default_waves_per_block = kOnchipWaves;
    r.default_flags = (int32_t)dflt_mask;
    r.candidates = (int32_t)cand.size();
    r.ms_per_generation = best->ms;
    r.default_ms_per_generation = dflt ? dflt->ms : -1.0;
    out->push_back(r);
    return QIEO_OK;
}

int Engine::tune_classes(int gens, std::vector<qieo_class_tune>* out)
{
    out->clear();
    int rc = ensure_built();
    if (rc) return rc;
    const size_t n = members_.size();
    if (n == 0 || (classes_.empty() && onchip_.empty())) return QIEO_OK;
    hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // the built-in rule's classes (the shapes a tuned entry replaces)
    std::vector<MemberShape> shapes(n);
    for (size_t i = 0; i < n; ++i) {
        const Member& m = members_[i];
        shapes[i] = MemberShape{m.np, m.L.pitch, m.L.nchunk, m.L.part_nseg,
                                (uint64_t)(uintptr_t)m.arena, m.window > 0, m.packed};
    }
    PlanOptions opt;
    opt.use_persistent = use_persistent_;
    opt.lds_limit = use_persistent_ ? resident_lds_limit() : 0;
    opt.use_segments = use_segments_;
    opt.merge_segments = merge_segments_;
    set_onchip_options(&opt);
    BatchPlan plan;
    if ((rc = plan_batch(shapes, opt, &plan))) return rc;
    // every member's state, saved once, restored before each candidate and
    // at the end
    std::vector<size_t> off(n + 1, 0);
    for (size_t i = 0; i < n; ++i) off[i + 1] = off[i] + (members_[i].L.total + 255) / 256 * 256;
    char* backup = (char*)mem_.alloc(off[n]);
    if (!backup) return set_error(QIEO_ENOMEM, "no device memory for a copy of the batch state");
    std::vector<void*> temps;           // tile tables of the candidates
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(stream_);
        for (void* p : temps) mem_.release(p);
        mem_.release(backup);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        dirty_ = true;                  // the next call rebuilds with the tuned shapes
        return code;
    };
    for (size_t i = 0; i < n && e == hipSuccess; ++i)
        e = hipMemcpyAsync(backup + off[i], members_[i].arena, members_[i].L.total,
                           hipMemcpyDeviceToDevice, stream_);
    for (size_t i = 0; i < n; ++i) h_gens_[i] = gens;
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_gens_, h_gens_, n * sizeof(int32_t), hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return done(hip_fail(e, "tuning set-up"));
    auto restore = [&](const std::vector<uint32_t>& ids) {
        hipError_t ee = hipSuccess;
        for (uint32_t i : ids) {
            if (ee != hipSuccess) break;
            ee = hipMemcpyAsync(members_[i].arena, backup + off[i], members_[i].L.total,
                                hipMemcpyDeviceToDevice, stream_);
        }
        return ee;
    };
    auto upload = [&](const std::vector<Tile>& t, Tile** d) {
        *d = (Tile*)mem_.alloc(t.size() * sizeof(Tile));
        if (!*d) return set_error(QIEO_ENOMEM, "device allocation of tuning tiles failed");
        temps.push_back(*d);
        const hipError_t ee = hipMemcpyAsync(*d, t.data(), t.size() * sizeof(Tile),
                                             hipMemcpyHostToDevice, stream_);
        return ee == hipSuccess ? QIEO_OK : hip_fail(ee, "hipMemcpyAsync(tiles)");
    };
    if (!plan.onchip.empty() && (rc = tune_onchip(gens, shapes, opt, plan, restore, temps, e0, e1,
                                                  out)))
        return done(rc);
    for (const ClassPlan& def : plan.classes) {
        // the class's members, longest rows first (as the planner orders them)
        std::vector<uint32_t> ids;
        if (def.flags & kFlagSegments) {
            for (const Tile& t : def.fe_tiles)
                if (ids.empty() || ids.back() != t.inst) ids.push_back(t.inst);
        } else {
            for (const Tile& t : def.tiles)
                if (ids.empty() || ids.back() != t.inst) ids.push_back(t.inst);
        }
        struct Cand {
            int R, S, flags;
            const Tile* tiles;
            int n_tiles;
            const Tile* fe;
            int n_fe;
            double ms;
        };
        std::vector<Cand> cand;
        // row order at rows per workgroup 1, 2, 4
        Tile* d_rows[3] = {nullptr, nullptr, nullptr};
        int n_rows[3] = {0, 0, 0};
        for (int ri = 0; ri < 3; ++ri) {
            const int R = 1 << ri;
            std::vector<Tile> t;
            for (uint32_t i : ids)
                for (int32_t r0 = 0; r0 < members_[i].np; r0 += R) t.push_back(Tile{i, (uint32_t)r0});
            if ((rc = upload(t, &d_rows[ri]))) return done(rc);
            n_rows[ri] = (int)t.size();
        }
        const int S0 = kClassWaves[def.cls];
        std::vector<int> waves;
        for (int S : {std::max(1, S0 / 2), S0, std::min(16, 2 * S0)})
            if (std::find(waves.begin(), waves.end(), S) == waves.end()) waves.push_back(S);
        for (int ri = 0; ri < 3; ++ri)
            for (int S : waves)
                for (int f = 0; f < 8; ++f)
                    cand.push_back(Cand{1 << ri, S, f, d_rows[ri], n_rows[ri], nullptr, 0, 1e300});
        if (def.flags & kFlagSegments) {
            Tile *d_seg = nullptr, *d_fe = nullptr;
            if ((rc = upload(def.tiles, &d_seg)) || (rc = upload(def.fe_tiles, &d_fe)))
                return done(rc);
            for (int f : {0, kFlagNontemporal, kFlagNontemporalLoads,
                          kFlagNontemporal | kFlagNontemporalLoads})
                cand.push_back(Cand{1, kSegWaves32, kFlagSegments | f, d_seg, (int)def.tiles.size(),
                                    d_fe, (int)def.fe_tiles.size(), 1e300});
        }
        auto time_one = [&](Cand& c) {
            hipError_t ee = restore(ids);
            if (ee == hipSuccess) ee = hipEventRecord(e0, stream_);
            for (int k = 0; k < gens && ee == hipSuccess; ++k)
                ee = (c.flags & kFlagSegments)
                         ? launch_segments_tiled(d_desc_, c.tiles, c.n_tiles, c.fe, c.n_fe,
                                                 c.flags, k, d_gens_, stream_)
                         : launch_generation(d_desc_, c.tiles, c.n_tiles, c.R, c.S, c.flags, k,
                                             d_gens_, 0, stream_);
            if (ee == hipSuccess) ee = hipEventRecord(e1, stream_);
            if (ee == hipSuccess) ee = hipEventSynchronize(e1);
            float ms = 0.f;
            if (ee == hipSuccess) ee = hipEventElapsedTime(&ms, e0, e1);
            if (ee != hipSuccess) return hip_fail(ee, "tuning launch");
            c.ms = std::min(c.ms, (double)ms / gens);
            return QIEO_OK;
        };
        for (int pass = 0; pass < 2; ++pass)
            for (size_t j = 0; j < cand.size(); ++j)
                if ((rc = time_one(cand[pass == 0 ? j : cand.size() - 1 - j]))) return done(rc);
        const Cand* best = &cand[0];
        const Cand* dflt = nullptr;
        for (const Cand& c : cand) {
            if (c.ms < best->ms) best = &c;
            // a segment-order launch ignores the row shape: its flags name it
            const bool same = (def.flags & kFlagSegments)
                                  ? c.flags == def.flags
                                  : c.R == def.R && c.S == def.S && c.flags == def.flags;
            if (same) dflt = &c;
        }
        record_class(def.cls, def.rows, def.max_nchunk, best->R, best->S, best->flags, best->ms);
        qieo_class_tune r{};
        r.shape_class = def.cls;
        r.rows = (int32_t)std::min<int64_t>(def.rows, INT32_MAX);
        r.max_chunks = def.max_nchunk;
        r.rows_per_block = best->R;
        r.waves_per_block = best->S;
        r.flags = best->flags;
        r.default_rows_per_block = def.R;
        r.default_waves_per_block = def.S;
        r.default_flags = def.flags;
        r.candidates = (int32_t)cand.size();
        r.ms_per_generation = best->ms;
        r.default_ms_per_generation = dflt ? dflt->ms : -1.0;
        out->push_back(r);
    }
    // the batch's own state back, as it was before tuning
    std::vector<uint32_t> all(n);
    for (size_t i = 0; i < n; ++i) all[i] = (uint32_t)i;
    if ((e = restore(all)) != hipSuccess) return done(hip_fail(e, "restore"));
    return done(QIEO_OK);
}

int Engine::set_window_all(int32_t window)
{
    for (auto& m : members_) {
        if (m.t != 0) return set_error(QIEO_ESTATE, "the convergence window is set before the first generation");
    }
    for (auto& m : members_) {
        int rc = write_window(m.d, stream_, window);
        if (rc) return rc;
        m.window = window;
    }
    // the batched on-chip launches are planned by window
    if (use_onchip_) dirty_ = true;
    return QIEO_OK;
}

}  // namespace qieo

// ---------------------------------------------------------------------------
// Batch C ABI
// ---------------------------------------------------------------------------
using namespace qieo;

struct qieo_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevicePool pool;
    Engine* eng = nullptr;
};

static void batch_release(qieo_batch* b)
{
    if (!b) return;
    delete b->eng;
    b->eng = nullptr;
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

extern "C" int qieo_batch_create(const qieo_problem* probs, int32_t n, const qieo_dev_ctx* ctx,
                                 qieo_batch** out)
{
    clear_error();
    if (!out) return set_error(QIEO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !probs) return set_error(QIEO_EINVAL, "need n >= 1 problems (got %d)", n);
    if (ctx && ((ctx->alloc == nullptr) != (ctx->free == nullptr)))
        return set_error(QIEO_EINVAL, "ctx->alloc and ctx->free must be both set or both NULL");
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        int rc = validate_problem(probs[i].items, probs[i].n_items, probs[i].capacity,
                                  probs[i].n_pop);
        if (rc) return set_error(rc, "problem %d: %s", i, qieo_last_error());
        ArenaLayout L;
        total += round256(arena_layout(probs[i].n_items, probs[i].n_pop, &L));
        // each arena is below 2^41 bytes, so the sum stops short of wrapping
        if (total > ((size_t)1 << 50))
            return set_error(QIEO_ENOMEM, "the batch needs more than 2^50 bytes of device memory");
    }
    int rc = check_device();
    if (rc) return rc;
    qieo_batch* b = new (std::nothrow) qieo_batch();
    if (!b) return set_error(QIEO_ENOMEM, "host allocation failed");
    hipError_t e;
    if (ctx && ctx->stream) {
        b->stream = (hipStream_t)ctx->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
            batch_release(b);
            return rc;
        }
        b->own_stream = true;
    }
    if ((rc = b->pool.init(total, ctx))) {
        batch_release(b);
        return rc;
    }
    b->eng = new (std::nothrow) Engine(b->stream, ctx);
    if (!b->eng) {
        batch_release(b);
        return set_error(QIEO_ENOMEM, "host allocation failed");
    }
    b->eng->set_use_onchip(true);
    for (int32_t i = 0; i < n; ++i) {
        if ((rc = b->eng->add(b->pool, probs[i].items, probs[i].n_items, probs[i].capacity,
                              probs[i].n_pop, probs[i].seed, (uint64_t)i, 0))) {
            batch_release(b);
            return rc;
        }
    }
    // descriptors, shape classes and tile tables of the initial membership
    if ((rc = b->eng->ensure_built())) {
        batch_release(b);
        return rc;
    }
    *out = b;
    return QIEO_OK;
}

extern "C" int qieo_batch_step_async(qieo_batch* b, const int32_t* n_gen_per_inst)
{
    clear_error();
    if (!b || !n_gen_per_inst) return set_error(QIEO_EINVAL, "NULL argument");
    return b->eng->run(n_gen_per_inst);
}

extern "C" int qieo_batch_sync(qieo_batch* b)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "NULL argument");
    return b->eng->sync();
}

extern "C" int qieo_batch_step(qieo_batch* b, const int32_t* n_gen_per_inst)
{
    int rc = qieo_batch_step_async(b, n_gen_per_inst);
    if (rc) return rc;
    return qieo_batch_sync(b);
}

extern "C" int qieo_batch_size(const qieo_batch* b, int32_t* n)
{
    clear_error();
    if (!b || !n) return set_error(QIEO_EINVAL, "NULL argument");
    *n = (int32_t)b->eng->size();
    return QIEO_OK;
}

static int batch_member(qieo_batch* b, int32_t i, Member** m)
{
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (i < 0 || (size_t)i >= b->eng->size())
        return set_error(QIEO_EINVAL, "instance %d outside [0, %zu)", i, b->eng->size());
    *m = &b->eng->member((size_t)i);
    return QIEO_OK;
}

extern "C" int qieo_batch_best(qieo_batch* b, int32_t i, qieo_result* out, uint32_t* bits,
                               size_t n_words)
{
    clear_error();
    Member* m;
    int rc = batch_member(b, i, &m);
    if (rc) return rc;
    if (!out) return set_error(QIEO_EINVAL, "out is NULL");
    return read_best(m->d, m->capacity, b->stream, out, bits, n_words);
}

extern "C" int qieo_batch_generations(qieo_batch* b, int32_t i, int64_t* out)
{
    clear_error();
    Member* m;
    int rc = batch_member(b, i, &m);
    if (rc) return rc;
    if (!out) return set_error(QIEO_EINVAL, "out is NULL");
    return read_generations(m->d, b->stream, out);
}

extern "C" int qieo_batch_set_convergence(qieo_batch* b, int32_t window)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (window < 0 || window > kConvRing)
        return set_error(QIEO_EINVAL, "window must be in [0, %d] (got %d)", kConvRing, window);
    return b->eng->set_window_all(window);
}

extern "C" int qieo_batch_converged(qieo_batch* b, int32_t i, int32_t* converged,
                                    int64_t* generation)
{
    clear_error();
    Member* m;
    int rc = batch_member(b, i, &m);
    if (rc) return rc;
    return read_convergence(m->d, b->stream, converged, generation);
}

extern "C" int qieo_batch_export_rows(qieo_batch* b, int32_t i, int32_t row0, int32_t n_rows,
                                      float* alpha, float* beta, uint8_t* alleles,
                                      int32_t* fitness, int32_t* profit, int32_t* weight,
                                      int32_t* elite)
{
    clear_error();
    Member* m;
    int rc = batch_member(b, i, &m);
    if (rc) return rc;
    int e = b->eng->sync();
    if (e) return e;
    // the descriptor array is rebuilt lazily; make sure it describes member i
    if ((e = b->eng->ensure_built())) return e;
    return export_rows(m->d, b->eng->device_desc((size_t)i), b->stream, row0, n_rows,
                       alpha, beta, alleles, fitness, profit, weight, elite);
}

extern "C" int qieo_batch_set_tile(qieo_batch* b, int32_t rows_per_block,
                                   int32_t waves_per_block, int32_t flags)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (rows_per_block == 0) {
        b->eng->force_shape(0, 0, 0);
        return QIEO_OK;
    }
    if ((rows_per_block != 1 && rows_per_block != 2 && rows_per_block != 4) ||
        waves_per_block < 1 || waves_per_block > 16 || flags < 0 || flags > kFlagAll ||
        (flags & kFlagSegments))
        return set_error(QIEO_EINVAL, "bad work shape (%d, %d, %d)", rows_per_block,
                         waves_per_block, flags);
    b->eng->force_shape(rows_per_block, waves_per_block, flags);
    return QIEO_OK;
}

extern "C" int qieo_batch_set_persistent(qieo_batch* b, int32_t enabled)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    b->eng->set_use_persistent(enabled != 0);
    return QIEO_OK;
}

extern "C" int qieo_batch_set_segment_order(qieo_batch* b, int32_t enabled)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (enabled < 0 || enabled > 2)
        return set_error(QIEO_EINVAL, "segment order mode must be 0, 1 or 2 (got %d)", enabled);
    b->eng->set_use_segments(enabled);
    return QIEO_OK;
}

extern "C" int qieo_batch_set_onchip(qieo_batch* b, int32_t enabled)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    b->eng->set_use_onchip(enabled != 0);
    return QIEO_OK;
}

extern "C" int qieo_batch_onchip_launches(qieo_batch* b, int32_t* n)
{
    clear_error();
    if (!b || !n) return set_error(QIEO_EINVAL, "NULL argument");
    int rc = b->eng->ensure_built();
    if (rc) return rc;
    *n = (int32_t)b->eng->onchip_launches();
    return QIEO_OK;
}

extern "C" int qieo_batch_set_barrier_timeout(qieo_batch* b, int64_t microseconds)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (microseconds < 0)
        return set_error(QIEO_EINVAL, "barrier timeout must be >= 0 (got %lld)",
                         (long long)microseconds);
    b->eng->set_barrier_us(microseconds);
    return QIEO_OK;
}

extern "C" int qieo_batch_autotune(qieo_batch* b, int32_t trial_generations,
                                   qieo_class_tune* out, int32_t max_out, int32_t* n_out)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    if (trial_generations < 1 || trial_generations > 1000)
        return set_error(QIEO_EINVAL, "trial_generations must be in [1, 1000] (got %d)",
                         trial_generations);
    if (max_out < 0 || (max_out > 0 && !out)) return set_error(QIEO_EINVAL, "bad output array");
    std::vector<qieo_class_tune> res;
    const int rc = b->eng->tune_classes(trial_generations, &res);
    if (rc) return rc;
    for (size_t i = 0; i < res.size() && (int32_t)i < max_out; ++i) out[i] = res[i];
    if (n_out) *n_out = (int32_t)res.size();
    return QIEO_OK;
}

extern "C" int qieo_batch_set_graph(qieo_batch* b, int32_t enabled)
{
    clear_error();
    if (!b) return set_error(QIEO_EINVAL, "batch is NULL");
    b->eng->set_use_graph(enabled != 0);
    return QIEO_OK;
}

extern "C" void qieo_batch_destroy(qieo_batch* b) { batch_release(b); }
