// Host-side planning of the library: arena layout, argument validation,
// work-shape rules, the offset allocator of a device pool, the batch's shape
// classes and tile tables, segment numbering constants and snapshot
// headers.  Plain C++ with no HIP call, so every piece here builds with a
// host compiler alone and is checked on the CPU (including under the
// address and undefined-behaviour sanitizers); the runtime, the batch
// engine and the server use these functions and add the device calls.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>
#include <vector>

#include "../../include/qieo.h"
#include "qieo_layout.hpp"

namespace qieo {

// ---- errors --------------------------------------------------------------
// Stores a thread-local message (read by qieo_last_error) and returns code.
int set_error(int code, const char* fmt, ...);
void clear_error();
const char* last_error();

// ---- arena ---------------------------------------------------------------
// Byte offsets of every plane inside one instance's device arena.
// part_nseg: segments per row the partial-sum array holds (segments of
// kSegChunksMin chunks); a segment-order launch must use no more.
struct ArenaLayout {
    int32_t pitch, nchunk;
    int32_t part_nseg;
    size_t alpha, beta, xbits, v, w, fit, prof, wt, ekey, best, best_bits, tbase, conv, sync, part;
    size_t zero_from;
    size_t total;
};

// elem: bytes per amplitude (4 binary32, 8 binary64); returns L->total.
// The shape must have passed validate_shape.
size_t arena_layout(int32_t ng, int32_t np, ArenaLayout* L, int elem = 4);
// True when a segment-order launch with segments of sc chunks stays inside
// the arena's partial-sum array.
bool segments_fit(const ArenaLayout& L, int sc);

// n_items in [1, 2^30 - 256], n_pop >= 1, at most 2^36 genes (rows padded to 64)
int validate_shape(int32_t n_items, int32_t n_pop);
int validate_problem(const qieo_item* items, int32_t n_items, int32_t capacity, int32_t n_pop);
// FNV-1a (64-bit) over the item array: identifies the problem a snapshot
// belongs to.
uint64_t items_fnv1a(const qieo_item* items, int32_t n);

// ---- work shapes ---------------------------------------------------------
// kFlag* bits for a work shape given the amplitude bytes one generation streams.
int variant_flags(int R, int S, int64_t nchunk, int64_t plane_bytes);
void pick_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags, int elem_bytes = 4);
// LDS bytes of the single-workgroup resident loop for one population.
size_t resident_lds_bytes(int32_t np, int32_t pitch, int32_t nchunk);

// ---- on-chip loop --------------------------------------------------------
// One cooperative launch runs every generation of a call with the amplitude
// planes held in registers: one workgroup of kOnchipWaves waves per CU,
// workgroup b owning rows [b*R, b*R + R) whole, wave w holding the
// workgroup's (row, chunk) items w*K .. w*K + K - 1 in row-major order, at
// 8 registers per item (a lane's four genes of alpha and beta).
constexpr int kOnchipWaves = 16;
// Shortest call the default mode runs this way.
constexpr int kOnchipMinGens = 4;
// Populations the default mode runs this way: a generation of the loop costs
// about 6 us however small the population (its synchronisation), while a
// per-generation launch costs 4.5-5.5 us for populations of up to ~128 rows
// and grows with the rows (6.2 us at 256, 9.5 at 512, 15 at 1024 rows of one
// chunk), so the loop pays from 256 rows, from 1024 (row, chunk) items, or
// from rows of 20 chunks, whose launches walk long chains of chunks per wave
// (measured over 25 shapes from 16 x 100 to 4096 x 1000).
bool onchip_worth(int32_t np, int32_t nchunk);
constexpr int kOnchipVariants = 5;
constexpr int kOnchipK[kOnchipVariants] = {2, 4, 6, 8, 10};   // compiled items per wave
struct OnchipPlan {
    bool packed = false;  // packed item tables (items_packable)
    int R = 0;          // rows per workgroup
    int blocks = 0;     // workgroups, at most one per CU
    int K = 0;          // items per wave: a compiled variant
    size_t lds = 0;     // dynamic LDS bytes per workgroup
    bool conv = false;  // the variant that makes the convergence-window test
                        // (set by the caller: the instance has a window)
};
// Item tables (one word per item when packed, else two), the workgroup's
// own allele words of two generations, the elite's words, and per row the
// fitness, profit and weight of two generations and the running sums.
size_t onchip_lds_bytes(int R, int32_t nchunk, bool packed = false);
// Packed item tables: every profit and weight of an instance in [0,
// kPackedItemMax] lets the on-chip loops keep one LDS word per item,
// profit | weight << 16; a lane's sum over its four genes then stays below
// 2^16 in each half, so one masked sum gives both exactly.
constexpr int32_t kPackedItemMax = (1 << 14) - 1;
bool items_packable(const qieo_item* items, int32_t n);
// False when the population does not fit: more items per wave than the
// largest variant, or more LDS than lds_limit.
bool onchip_plan(int32_t np, int32_t nchunk, int n_cu, size_t lds_limit, OnchipPlan* out,
                 bool packed = false);

// Segment numbering constants of one segment-order launch of n_seg
// workgroups on a device of `xcds` XCDs; nseg_row > 0 for an untiled launch
// (segments per row of its single instance), 0 for a tiled one.
SegMap seg_map_for(int64_t n_seg, int xcds, int32_t nseg_row);

// ---- device pool bookkeeping --------------------------------------------
// First-fit offset allocator over [0, capacity): blocks are 256-byte
// aligned; freed ranges coalesce with their neighbours.
class OffsetAllocator {
public:
    static constexpr size_t npos = (size_t)-1;
    void reset(size_t capacity);               // capacity rounded up to 256
    size_t alloc(size_t bytes);                // offset, or npos if no room
    bool release(size_t offset);               // false if not a live block
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const;
    size_t live_blocks() const { return busy_.size(); }
    // Consistency of the free and busy maps (tests): disjoint, sorted,
    // coalesced, 256-aligned, covering [0, capacity) exactly.
    bool check() const;

private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    std::map<size_t, size_t> busy_;   // offset -> size
};

// ---- batch shape classes -------------------------------------------------
// Shape classes by 256-gene chunks per row: 1, 2-3, 4-7, 8-31, >= 32; the
// class's waves per workgroup are 1, 2, 4, 8, 16.
constexpr int kClasses = 5;
constexpr int kClassWaves[kClasses] = {1, 2, 4, 8, 16};
// Largest segment tile table a class keeps (32 MB of tiles).
constexpr int64_t kMaxSegTiles = (int64_t)1 << 22;
int class_of(int32_t nchunk);

// What the planner needs to know of one member of a batch.
struct MemberShape {
    int32_t np = 0, pitch = 0, nchunk = 0;
    int32_t part_nseg = 0;        // from the member's arena layout
    uint64_t addr = 0;            // arena address (segment tiles go in address order)
    bool conv = false;            // has a convergence window
    bool packed = false;          // items_packable
};

struct PlanOptions {
    bool use_persistent = true;   // LDS-resident members as single workgroups
    size_t lds_limit = 0;         // dynamic LDS the resident kernel may take
    // Batched on-chip loop for every member it can place (before the
    // LDS-resident set and the classes): workgroups per launch (the
    // device's CUs; 0 = off), the dynamic LDS a workgroup may take, and the
    // usable compiled variants (bit v: kOnchipK[v]).
    int onchip_blocks = 0;
    size_t onchip_lds_limit = 0;
    unsigned onchip_variants = 0;
    bool use_segments = true;     // long rows in segment order when the batch streams
    bool merge_segments = true;   // rows of 8+ chunks in one segment table
    int force_R = 0, force_S = 0, force_flags = 0;   // every class, when force_R > 0
    // Tuned shapes: the autotuner's entry for (class, rows of the class,
    // longest row in chunks), or NULL.
    bool (*tuned)(int cls, int64_t rows, int32_t max_nchunk, int* R, int* S, int* flags) = nullptr;
};

// One launch class of a batch.  Row order: tiles {member, first row}, R
// rows each.  Segment order (flags has kFlagSegments): tiles {member,
// segment number} in arena address order, fe_tiles {member, first of four
// rows}.
struct ClassPlan {
    int cls = 0;                  // shape class (0 .. kClasses-1)
    int R = 1, S = 1, flags = 0;
    bool tuned = false;           // shape from the tuning database
    int64_t rows = 0;
    int32_t max_nchunk = 0;
    std::vector<Tile> tiles, fe_tiles;
};

// One workgroup of a batched on-chip launch: rows [row0, row0 + nrows) of
// member inst, which the launch runs on nb workgroups (blk = this one's
// index among them) of up to R rows each.
struct OnchipTile {
    uint32_t inst;
    int32_t row0, nrows, R;
    int32_t blk, nb;
    int32_t pad[2];
};

// One cooperative launch of the batched on-chip loop: every generation of
// the call for the members its tiles cover, one workgroup per tile.
struct OnchipLaunch {
    int K = 0;                        // compiled items per wave
    bool conv = false;                // the variant with the window test (its members have windows)
    bool packed = false;              // the variant with packed item tables (its members' items fit)
    size_t lds = 0;                   // dynamic LDS per workgroup (the largest tile's need)
    std::vector<OnchipTile> tiles;
};

struct BatchPlan {
    std::vector<uint32_t> resident;   // members run by the LDS-resident kernel, largest first
    size_t resident_lds = 0;          // its dynamic LDS (the largest member's need)
    std::vector<OnchipLaunch> onchip; // batched on-chip launches, run one after another
    std::vector<ClassPlan> classes;   // smallest rows first
};

// Places members (indices into `members`) on batched on-chip launches.
// Each member takes the usable variant K that costs it least, counted as
// its workgroups times the measured cost of a workgroup-generation (about 6
// us of synchronisation plus 1.1 us per item a wave holds): at variant K it
// runs on b workgroups of R = ceil(np / b) whole rows, b the fewest whose
// kOnchipWaves * K items hold its rows.  The members of each variant, those
// with a convergence window apart from those without and those with packed
// item tables apart from the others, are packed first-fit
// by decreasing b into launches of at most opt.onchip_blocks workgroups;
// then each launch whose members all fit the spare workgroups of launches
// of a larger variant (their b recomputed there) is emptied into them,
// cheapest launches first.  Members no variant can place (a row longer
// than the largest variant holds, more workgroups than a launch has, more
// LDS than the limit, more than 65536 rows) are returned in *rest.
void plan_onchip(const std::vector<MemberShape>& members, const std::vector<size_t>& ids,
                 const PlanOptions& opt, std::vector<OnchipLaunch>* out, std::vector<size_t>* rest);

// Groups members into the resident set and the shape classes and builds
// every tile table.  QIEO_EINVAL if a table would not fit a launch or a
// member's arena cannot hold its segment sums.
int plan_batch(const std::vector<MemberShape>& members, const PlanOptions& opt, BatchPlan* out);

// ---- snapshots -----------------------------------------------------------
struct StateHeader {
    char magic[8];
    uint32_t version;
    uint32_t elem_bytes;
    int32_t n_items, n_pop, capacity, reserved;
    uint64_t seed;
    uint64_t items_hash;
    int64_t generations;
    uint64_t arena_bytes;
};

// Identity of the handle a snapshot is loaded into.
struct SnapshotId {
    uint32_t elem_bytes;
    int32_t n_items, n_pop, capacity;
    uint64_t seed, items_hash;
};

StateHeader make_state_header(const SnapshotId& id, int64_t generations, uint64_t arena_bytes);
// Checks a snapshot buffer (header plus arena image) against the handle's
// identity and layout before anything is copied to the device: magic and
// version, precision, problem, size, and the image's own generation
// counter, convergence window and latest elite row.  On success returns
// QIEO_OK with the image's generation count and window; else QIEO_EINVAL.
int check_snapshot(const void* buf, size_t bytes, const SnapshotId& id, const ArenaLayout& L,
                   int64_t* generations, int32_t* window);

}  // namespace qieo
