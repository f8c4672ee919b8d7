// Multi-instance engine: many resident populations advanced together, one
// fused generation launch per shape class per generation, captured in a HIP
// graph.  Used by the batch API and by the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <vector>

#include "qieo_internal.hpp"

namespace qieo {

// First-fit offset allocator over one device allocation (the HBM budget of a
// server, or the exact total of a batch).  Blocks are 256-byte aligned; freed
// ranges are coalesced with their neighbours.
class DevicePool {
public:
    DevicePool() = default;
    ~DevicePool();
    int init(size_t bytes, const qieo_dev_ctx* ctx);   // QIEO_OK / QIEO_ENOMEM
    char* alloc(size_t bytes);                         // nullptr if no room
    void release(char* p);
    size_t capacity() const { return book_.capacity(); }
    size_t used() const { return book_.used(); }
    size_t largest_free() const { return book_.largest_free(); }

private:
    char* base_ = nullptr;
    DevMem mem_;
    OffsetAllocator book_;            // which byte ranges of the pool are in use
};

// One resident population inside an engine.
struct Member {
    InstDev d{};          // device pointers into its arena
    ArenaLayout L{};
    char* arena = nullptr;
    int32_t ng = 0, np = 0, capacity = 0;
    uint64_t seed = 0;
    int64_t t = 0;        // generations completed (host mirror; exact after refresh_status)
    uint64_t id = 0;      // caller's identifier
    int32_t window = 0;   // convergence window (0 = fixed budget)
    bool converged = false;
    bool packed = false;  // profits and weights fit the on-chip loops' packed item tables
};

// Work shape of one launch class.
struct ShapeClass {
    int cls = 0;               // shape class by chunks per row (class_of)
    int R = 4, S = 8, flags = 0;
    bool tuned = false;        // shape taken from the tuning database
    std::vector<Tile> tiles;
    Tile* d_tiles = nullptr;   // device copy
    // segment order (flags has kFlagSegments): tiles are {member, segment
    // number} in address order, fe_tiles {member, first of four rows}
    std::vector<Tile> fe_tiles;
    Tile* d_fe_tiles = nullptr;
};

class Engine {
public:
    // ctx: the caller's allocator (and stream) for the engine's own tables,
    // or NULL for hipMalloc
    Engine(hipStream_t s, const qieo_dev_ctx* ctx) : stream_(s) { mem_.set(ctx); }
    ~Engine();

    // Membership.  add() uploads items and initialises the state on the
    // engine's stream; the arena comes from `pool`.
    int add(DevicePool& pool, const qieo_item* items, int32_t n_items, int32_t capacity,
            int32_t n_pop, uint64_t seed, uint64_t id, int32_t window);
    void remove_at(size_t idx, DevicePool& pool);
    size_t size() const { return members_.size(); }
    Member& member(size_t i) { return members_[i]; }
    const InstDev* device_desc(size_t i) const { return d_desc_ + i; }

    // Runs gens[i] generations of member i (all members in the same launches)
    // and the finishing step; enqueued on the stream, not waited for.
    int run(const int32_t* gens);
    int sync();
    // Reads every member's generation counter and converged flag as left by
    // the last finished call (waits for the stream).
    int refresh_status();
    int set_window_all(int32_t window);

    // Shape-class override for experiments and tuning: every class uses
    // (R, S, flags) when R > 0.
    void force_shape(int R, int S, int flags);
    void set_use_graph(bool on) { use_graph_ = on; invalidate_graph(); }
    void set_use_persistent(bool on) { use_persistent_ = on; dirty_ = true; }
    // Batched on-chip loop for members of rows under 32 chunks (off by default)
    void set_use_onchip(bool on) { use_onchip_ = on; dirty_ = true; }
    bool use_onchip() const { return use_onchip_; }
    // On-chip launches the current plan makes per call (after ensure_built)
    size_t onchip_launches() const { return onchip_.size(); }
    // Bound on one on-chip barrier wait, in microseconds
    void set_barrier_us(int64_t us) { barrier_us_ = us; }
    // mode 0: row order everywhere; 1: segment order for rows of >= 8 chunks
    // of a streaming batch; 2: only for rows of >= 32 chunks
    void set_use_segments(int mode)
    {
        use_segments_ = mode != 0;
        merge_segments_ = mode == 1;
        dirty_ = true;
    }
    // Uploads descriptors and tile tables if membership changed since the
    // last launch (device_desc() is valid only after this).
    int ensure_built() { return dirty_ ? rebuild() : QIEO_OK; }

    // Times candidate work shapes for every launch class of the current
    // membership (gens generations each, every candidate from the same state:
    // the members' arenas are saved first and restored after each candidate
    // and at the end, so the batch's own trajectory does not move), records
    // the fastest per class in the tuning database and rebuilds the classes
    // with them.  out receives one entry per class.
    int tune_classes(int gens, std::vector<qieo_class_tune>* out);

private:
    int rebuild();               // descriptors and tile tables after membership change
    bool capture(int nmax);
    int enqueue(int nmax);
    void invalidate_graph();

    hipStream_t stream_;
    DevMem mem_;
    std::vector<Member> members_;
    bool dirty_ = true;
    InstDev* d_desc_ = nullptr;
    size_t desc_cap_ = 0;
    int32_t* d_gens_ = nullptr;
    int64_t* d_status_ = nullptr;  // per member {generations completed, converged}
    int32_t* h_gens_ = nullptr;    // pinned
    size_t gens_cap_ = 0;
    std::vector<ShapeClass> classes_;
    // small members: one persistent workgroup each, on a side stream forked
    // from and joined back into the main one
    std::vector<uint32_t> pids_;     // members run by the LDS-resident kernel
    size_t pids_lds_ = 0;            // its dynamic LDS (the largest member's need)
    uint32_t* d_pids_ = nullptr;
    hipStream_t side_ = nullptr;
    hipEvent_t fork_ = nullptr, join_ = nullptr;
    // batched on-chip launches (run first, on the main stream, before the
    // fork: each takes one workgroup on every CU it uses for the whole call)
    struct OnchipRun {
        int K = 0;
        bool conv = false;
        bool packed = false;
        size_t lds = 0;
        int n_tiles = 0;
        OnchipTile* d_tiles = nullptr;
    };
    std::vector<OnchipRun> onchip_;
    uint32_t* d_abort_ = nullptr;    // one abort word per on-chip launch
    bool onchip_check_ = false;      // launches queued since the abort words were read
    int check_onchip_abort();
    int tune_onchip(int gens, const std::vector<MemberShape>& shapes, const PlanOptions& opt,
                    const BatchPlan& plan,
                    const std::function<hipError_t(const std::vector<uint32_t>&)>& restore,
                    std::vector<void*>& temps, hipEvent_t e0, hipEvent_t e1,
                    std::vector<qieo_class_tune>* out);
    unsigned onchip_mask_ = 0;       // variant subset the tuner chose (0: every usable one)
    int device_of_stream() const;
    void batch_signature(int64_t* rows, int32_t* max_nchunk) const;
    void set_onchip_options(PlanOptions* opt) const;
    bool use_onchip_ = false;
    int64_t barrier_us_ = 1000000;
    // shape classes after the first run on streams of their own
    std::vector<hipStream_t> cstreams_;
    std::vector<hipEvent_t> cjoin_;
    bool use_persistent_ = true;
    bool use_segments_ = true;   // long rows in segment order when the batch streams
    bool merge_segments_ = true;
    int force_R_ = 0, force_S_ = 0, force_flags_ = 0;
    bool use_graph_ = true;
    bool use_tuned_ = true;      // class shapes from the tuning database where tuned
    hipGraphExec_t graph_ = nullptr;
    int graph_n_ = -1;
    int prev_n_ = -1;            // longest count of the previous call since the last rebuild
    std::vector<int32_t> staging_;
};

}  // namespace qieo
