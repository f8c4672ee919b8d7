// Checks of the library's host-only planning code (csrc/qieo_host.cpp),
// built by tests/test_host_sanitized.py with g++ under the address and
// undefined-behaviour sanitizers and run on the CPU.  Exit status 0 when
// every check passes; the first failure is printed and exits 1.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2609_30862_amd/csrc/qieo_host.hpp"

using namespace qieo;

static int g_checks = 0;

#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        ++g_checks;                                                          \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                               \
            std::fprintf(stderr, "\n");                                      \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// Arena layout and the segment sums' sizing
// ---------------------------------------------------------------------------
static void check_arena()
{
    const int32_t shapes[][2] = {{1, 1},       {3, 1},          {63, 5},       {64, 7},
                                 {65, 2},      {255, 3},        {256, 1},      {257, 9},
                                 {1000, 33},   {4097, 16},      {10000, 1024}, {200000, 4096},
                                 {20000, 1},   {131136, 32768}, {(1 << 30) - 256, 2},
                                 {50, 70001}};
    for (auto& sh : shapes) {
        const int32_t ng = sh[0], np = sh[1];
        CHECK(validate_shape(ng, np) == QIEO_OK, "shape %d x %d rejected", ng, np);
        for (int elem : {4, 8}) {
            ArenaLayout L;
            const size_t total = arena_layout(ng, np, &L, elem);
            CHECK(total == L.total, "total");
            CHECK(L.pitch >= ng && L.pitch % 64 == 0 && L.pitch - ng < 64, "pitch %d", L.pitch);
            CHECK(L.nchunk == (L.pitch + kChunk - 1) / kChunk, "nchunk");
            const size_t wpr = (size_t)L.nchunk * kWordsPerChunk;
            // every block 256-byte aligned, in order, disjoint, sized as stated
            struct B { size_t off, bytes; const char* name; };
            const B blocks[] = {
                {L.alpha, ((size_t)np * L.pitch + kChunk) * elem, "alpha"},
                {L.beta, ((size_t)np * L.pitch + kChunk) * elem, "beta"},
                {L.xbits, 2 * (size_t)np * wpr * 4, "xbits"},
                {L.v, (size_t)L.nchunk * kChunk * 4, "v"},
                {L.w, (size_t)L.nchunk * kChunk * 4, "w"},
                {L.fit, 2 * (size_t)np * 4, "fit"},
                {L.prof, 2 * (size_t)np * 4, "prof"},
                {L.wt, 2 * (size_t)np * 4, "wt"},
                {L.ekey, 24, "ekey"},
                {L.best, 32, "best"},
                {L.best_bits, wpr * 4, "best_bits"},
                {L.tbase, 8, "tbase"},
                {L.conv, 256, "conv"},
                {L.sync, 64 + 16 * (size_t)std::min(np, (int32_t)kOnchipMaxBlocks), "sync"},
                {L.part, (size_t)L.part_nseg * np * 8, "part"}};
            size_t end = 0;
            for (const B& b : blocks) {
                CHECK(b.off % 256 == 0, "%s misaligned", b.name);
                CHECK(b.off >= end, "%s overlaps the block before it", b.name);
                end = b.off + b.bytes;
            }
            CHECK(end <= L.total && L.total - end < 256, "total %zu, end %zu", L.total, end);
            // the part array holds the segments of every launch geometry
            CHECK(L.part_nseg == seg_count(L.nchunk, kSegChunksMin), "part_nseg");
            CHECK(segments_fit(L, kSegChunks32) && segments_fit(L, kSegChunks64),
                  "built-in segment geometry does not fit %d x %d", ng, np);
            // a shorter segment than the sizing needs more entries per row
            // whenever the row has more than one segment of the sizing
            if (L.nchunk > 1)
                CHECK(!segments_fit(L, 1), "1-chunk segments fit %d x %d", ng, np);
            // the last segment-order write of a launch with segments of sc
            // chunks: part[(np - 1) * nseg + nseg - 1] (two words)
            const size_t part_end = L.part + (size_t)L.part_nseg * np * 8;
            for (int sc = 1; sc <= 64; sc *= 2) {
                const int64_t nseg = seg_count(L.nchunk, sc);
                const size_t last = L.part + ((size_t)np * nseg) * 8;   // one past the end
                if (segments_fit(L, sc))
                    CHECK(last <= part_end && part_end <= L.total, "fits, yet past the end, sc %d", sc);
                else
                    CHECK(last > part_end, "refused although within the array, sc %d", sc);
            }
        }
    }
}

// A segment-order launch whose segments are shorter than the arena's sizing
// writes past the end of the arena (the part array is its last block).  The
// case of the sizing of 8-chunk segments (the binary32 geometry when the
// sizing took the shorter of the two precisions' segments, 8 and 16 chunks)
// launched with 4-chunk segments at 4096 x 200,000: 196 segments per row
// against 98, so the launch writes 3.2 MB past the arena's last byte.
static void check_historical_overflow()
{
    const int32_t ng = 200000, np = 4096;
    ArenaLayout L;
    arena_layout(ng, np, &L, 8);
    const int64_t sized = seg_count(L.nchunk, 8), launched = seg_count(L.nchunk, 4);
    CHECK(sized == 98 && launched == 196, "segments %lld %lld", (long long)sized,
          (long long)launched);
    const size_t part_then = (size_t)sized * np * 8;          // bytes the arena held
    const size_t written = (size_t)launched * np * 8;         // bytes the launch wrote
    CHECK(written - part_then == 3211264, "overflow %zu", written - part_then);
    // with today's sizing the same launch fits, and the helper says so
    CHECK(segments_fit(L, 4), "4-chunk segments must fit");
    CHECK(!segments_fit(L, 2) && !segments_fit(L, 1), "2-chunk segments must not fit");
}

// ---------------------------------------------------------------------------
// Segment numbering: XCD renumbering is a bijection, the row reciprocal is
// exact
// ---------------------------------------------------------------------------
static void check_seg_map()
{
    std::mt19937_64 rng(7);
    for (int xcds : {1, 2, 3, 4, 5, 6, 7, 8, 12, 16}) {
        for (int64_t n : {1ll, 2ll, 7ll, 8ll, 9ll, 63ll, 64ll, 65ll, 1000ll, 4097ll, 802816ll}) {
            const SegMap m = seg_map_for(n, xcds, 0);
            CHECK(m.q * (int64_t)m.xcds + m.r == n, "split of %lld over %d", (long long)n, xcds);
            std::vector<uint8_t> seen((size_t)n, 0);
            for (int64_t b = 0; b < n; ++b) {
                const int32_t s = seg_renumber(m, (int32_t)b);
                CHECK(s >= 0 && s < n, "renumbered %lld -> %d of %lld", (long long)b, s,
                      (long long)n);
                CHECK(!seen[(size_t)s], "%d taken twice", s);
                seen[(size_t)s] = 1;
                // workgroup b runs on XCD b mod xcds: its numbers form one run
                const int64_t x = b % m.xcds;
                const int64_t lo = x * m.q + std::min<int64_t>(x, m.r);
                const int64_t len = m.q + (x < m.r ? 1 : 0);
                CHECK(s >= lo && s < lo + len, "XCD %lld run", (long long)x);
            }
        }
    }
    // s / nseg by multiply and shift, exact for every s < 2^31
    std::vector<int32_t> nsegs = {1, 2, 3, 4, 5, 7, 49, 98, 196, 782, 1000, 1023, 1024, 1025,
                                  65535, 65536, 262143, 1048575, 4194303, 4194304, (1 << 30) - 1,
                                  (1 << 30), 2147483647};
    for (int k = 0; k < 40; ++k) nsegs.push_back((int32_t)(1 + rng() % 2147483647ull));
    for (int32_t nseg : nsegs) {
        const SegMap m = seg_map_for(1, 8, nseg);
        auto ok = [&](uint32_t s) {
            CHECK(seg_row(m, s) == (int32_t)(s / (uint32_t)nseg), "s %u / nseg %d", s, nseg);
        };
        for (uint32_t s = 0; s < 4096; ++s) ok(s);
        for (uint32_t s = 2147483647u - 4096; s < 2147483648u; ++s) ok(s);
        // around every multiple of nseg near sampled positions
        for (int k = 0; k < 2000; ++k) {
            const uint64_t q = rng() % (2147483648ull / (uint64_t)nseg + 1);
            for (int64_t d = -2; d <= 1; ++d) {
                const int64_t s = (int64_t)q * nseg + d;
                if (s >= 0 && s < 2147483648ll) ok((uint32_t)s);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Offset allocator against a byte-map model, with exhaustion
// ---------------------------------------------------------------------------
static void check_offset_allocator()
{
    std::mt19937_64 rng(11);
    for (int round = 0; round < 40; ++round) {
        const size_t cap = 256 * (1 + rng() % 512);
        OffsetAllocator a;
        a.reset(cap);
        CHECK(a.capacity() == cap && a.used() == 0 && a.check(), "fresh pool");
        std::vector<uint8_t> model(cap / 256, 0);
        std::map<size_t, size_t> live;
        for (int op = 0; op < 3000; ++op) {
            if (live.empty() || rng() % 3) {
                const size_t want = 1 + rng() % (cap / 4 + 1);
                const size_t units = (want + 255) / 256;
                // first fit on the model
                size_t run = 0, first = OffsetAllocator::npos;
                for (size_t u = 0; u < model.size(); ++u) {
                    run = model[u] ? 0 : run + 1;
                    if (run == units) { first = (u + 1 - units) * 256; break; }
                }
                const size_t off = a.alloc(want);
                CHECK(off == first, "alloc %zu: got %zu, first fit %zu", want, off, first);
                if (off != OffsetAllocator::npos) {
                    for (size_t u = off / 256; u < off / 256 + units; ++u) model[u] = 1;
                    live[off] = units;
                }
            } else {
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                CHECK(a.release(it->first), "release of a live block");
                CHECK(!a.release(it->first), "double release accepted");
                for (size_t u = it->first / 256; u < it->first / 256 + it->second; ++u) model[u] = 0;
                live.erase(it);
            }
            CHECK(a.check(), "inconsistent maps after op %d", op);
            size_t used = 0;
            for (auto& l : live) used += l.second * 256;
            CHECK(a.used() == used, "used %zu vs %zu", a.used(), used);
            CHECK(a.live_blocks() == live.size(), "live blocks");
        }
        for (auto& l : live) CHECK(a.release(l.first), "final release");
        CHECK(a.used() == 0 && a.largest_free() == cap && a.check(), "pool not whole again");
        CHECK(a.alloc(cap + 1) == OffsetAllocator::npos, "over-capacity request granted");
        CHECK(a.alloc(cap) == 0 && a.alloc(1) == OffsetAllocator::npos, "exhaustion");
        CHECK(!a.release(12345), "release of an unknown offset accepted");
    }
}

// ---------------------------------------------------------------------------
// Batch planning: every row (or segment) of every member in exactly one tile
// ---------------------------------------------------------------------------
static bool g_tuned_called = false;
static bool tuned_stub(int cls, int64_t, int32_t, int* R, int* S, int* F)
{
    g_tuned_called = true;
    if (cls != 2) return false;
    *R = 2;
    *S = 2;
    *F = kFlagPrefetch;
    return true;
}

static void check_plan_batch()
{
    std::mt19937_64 rng(5);
    for (int round = 0; round < 60; ++round) {
        const int n = 1 + (int)(rng() % 80);
        std::vector<MemberShape> ms(n);
        uint64_t addr = 1 << 20;
        std::vector<int32_t> ngs(n);
        for (int i = 0; i < n; ++i) {
            const int32_t ng = 1 + (int32_t)(rng() % (round % 3 == 0 ? 300000 : 20000));
            const int32_t np = 1 + (int32_t)(rng() % (round % 4 == 0 ? 2048 : 256));
            ArenaLayout L;
            arena_layout(ng, np, &L);
            ms[i].np = np;
            ms[i].pitch = L.pitch;
            ms[i].nchunk = L.nchunk;
            ms[i].part_nseg = L.part_nseg;
            ms[i].addr = addr + (uint64_t)(rng() % 1000) * 4096;   // not in member order
            ms[i].conv = rng() % 3 == 0;
            ms[i].packed = rng() % 2 == 0;
            addr += L.total + (1 << 20);
            ngs[i] = ng;
        }
        PlanOptions opt;
        opt.use_persistent = round % 2 == 0;
        opt.lds_limit = 160 * 1024 - 1024;
        opt.use_segments = round % 5 != 1;
        opt.merge_segments = round % 3 != 2;
        if (round % 7 == 3) { opt.force_R = 4; opt.force_S = 8; opt.force_flags = 3; }
        if (round % 7 == 5) opt.tuned = tuned_stub;
        if (round % 2 == 1) {
            // batched on-chip loop: a full device, or a small one that forces
            // several launches and leaves members with too many rows out
            opt.onchip_blocks = round % 4 == 1 ? 256 : 24;
            opt.onchip_lds_limit = round % 8 == 3 ? 6 * 1024 : 160 * 1024 - 256;
            opt.onchip_variants = round % 3 == 0 ? 0x1fu : 0x06u;
        }
        BatchPlan plan;
        CHECK(plan_batch(ms, opt, &plan) == QIEO_OK, "plan failed: %s", last_error());
        int64_t plane_bytes = 0;
        for (auto& m : ms) plane_bytes += (int64_t)m.np * m.pitch * 8;
        const bool streaming = opt.use_segments && opt.force_R == 0 && plane_bytes > (256ll << 20);
        // coverage: rows[i][r] counts tiles covering row r of member i;
        // segs[i] counts segment tiles by segment number
        std::vector<std::vector<int>> rows(n), fe(n), segs(n);
        std::vector<int> where(n, -1);
        for (int i = 0; i < n; ++i) {
            rows[i].assign(ms[i].np, 0);
            fe[i].assign(ms[i].np, 0);
        }
        for (uint32_t id : plan.resident) {
            CHECK(id < (uint32_t)n && where[id] == -1, "resident id %u", id);
            CHECK(opt.use_persistent &&
                      resident_lds_bytes(ms[id].np, ms[id].pitch, ms[id].nchunk) <= opt.lds_limit,
                  "member %u resident without fitting", id);
            where[id] = 100;
            for (auto& r : rows[id]) r = 1;
            for (auto& r : fe[id]) r = 1;
        }
        CHECK((opt.onchip_blocks > 0 && opt.force_R == 0) || plan.onchip.empty(),
              "on-chip launches while off or under a forced shape");
        for (const OnchipLaunch& L : plan.onchip) {
            int v = 0;
            while (v < kOnchipVariants && kOnchipK[v] != L.K) ++v;
            CHECK(v < kOnchipVariants && (opt.onchip_variants >> v & 1u), "variant K %d", L.K);
            CHECK(!L.tiles.empty() && (int)L.tiles.size() <= opt.onchip_blocks,
                  "%zu workgroups in a launch of at most %d", L.tiles.size(), opt.onchip_blocks);
            size_t lds = 0;
            std::map<uint32_t, std::vector<int>> blk_seen;
            for (const OnchipTile& t : L.tiles) {
                CHECK(t.inst < (uint32_t)n, "on-chip tile member");
                const MemberShape& m = ms[t.inst];
                CHECK(m.conv == L.conv, "member %u (window %d) in a launch with window test %d",
                      t.inst, (int)m.conv, (int)L.conv);
                CHECK(m.packed == L.packed, "member %u (packed %d) in a launch with packed %d",
                      t.inst, (int)m.packed, (int)L.packed);
                CHECK(m.np <= 65536, "member %u: %d rows on-chip", t.inst, m.np);
                CHECK(t.nb >= 1 && t.nb <= opt.onchip_blocks && t.blk >= 0 && t.blk < t.nb,
                      "workgroup %d of %d", t.blk, t.nb);
                CHECK(t.R >= 1 && (int64_t)t.R * m.nchunk <= (int64_t)kOnchipWaves * L.K,
                      "R %d x %d chunks beyond %d items", t.R, m.nchunk, kOnchipWaves * L.K);
                CHECK(t.row0 == t.blk * t.R && t.nrows == std::min(t.R, m.np - t.row0) &&
                          t.nrows >= 1,
                      "rows %d + %d of member %u", t.row0, t.nrows, t.inst);
                CHECK((int64_t)t.nb == ((int64_t)m.np + t.R - 1) / t.R, "nb %d", t.nb);
                auto& seen = blk_seen[t.inst];
                if (seen.empty()) {
                    CHECK(where[t.inst] == -1, "member %u in two on-chip launches", t.inst);
                    seen.assign(t.nb, 0);
                    where[t.inst] = 200;
                }
                CHECK((int)seen.size() == t.nb && ++seen[t.blk] == 1, "workgroup %d repeated", t.blk);
                for (int32_t r = t.row0; r < t.row0 + t.nrows; ++r) {
                    rows[t.inst][r]++;
                    fe[t.inst][r]++;
                }
                lds = std::max(lds, onchip_lds_bytes(t.R, m.nchunk, m.packed));
            }
            CHECK(L.lds == lds && lds <= opt.onchip_lds_limit, "launch LDS %zu (tiles %zu)", L.lds,
                  lds);
        }
        int prev_cls = -1;
        for (const ClassPlan& c : plan.classes) {
            CHECK(c.cls > prev_cls, "classes out of order");
            prev_cls = c.cls;
            CHECK(c.R == 1 || c.R == 2 || c.R == 4, "R %d", c.R);
            CHECK(c.S >= 1 && c.S <= 16, "S %d", c.S);
            const bool seg = (c.flags & kFlagSegments) != 0;
            if (seg) {
                CHECK(streaming && c.cls == kClasses - 1, "segment order outside a streaming long-row class");
                uint64_t last_addr = 0;
                uint32_t last_inst = UINT32_MAX;
                for (const Tile& t : c.tiles) {
                    CHECK(t.inst < (uint32_t)n, "tile member");
                    const MemberShape& m = ms[t.inst];
                    const int64_t nseg = seg_count(m.nchunk, kSegChunks32);
                    CHECK((int64_t)t.row0 < (int64_t)m.np * nseg, "segment number");
                    if (t.inst != last_inst) {
                        CHECK(m.addr >= last_addr, "segment tiles not in address order");
                        last_addr = m.addr;
                        last_inst = t.inst;
                        CHECK(segs[t.inst].empty(), "member %u split", t.inst);
                        segs[t.inst].assign((size_t)((int64_t)m.np * nseg), 0);
                        where[t.inst] = c.cls;
                    }
                    segs[t.inst][t.row0]++;
                    rows[t.inst][t.row0 / nseg] = 1;
                }
                for (const Tile& t : c.fe_tiles) {
                    CHECK(t.inst < (uint32_t)n && t.row0 % 4 == 0, "fe tile");
                    for (uint32_t r = t.row0; r < std::min<uint32_t>(t.row0 + 4, ms[t.inst].np); ++r)
                        fe[t.inst][r]++;
                }
            } else {
                CHECK(c.fe_tiles.empty(), "row order with closing tiles");
                if (opt.force_R) {
                    CHECK(c.R == opt.force_R && c.S == opt.force_S && c.flags == opt.force_flags,
                          "forced shape not used");
                } else if (c.tuned) {
                    CHECK(c.cls == 2 && c.R == 2 && c.S == 2, "tuned shape");
                }
                for (const Tile& t : c.tiles) {
                    CHECK(t.inst < (uint32_t)n, "tile member");
                    CHECK(where[t.inst] == -1 || where[t.inst] == c.cls, "member in two classes");
                    where[t.inst] = c.cls;
                    CHECK(t.row0 % c.R == 0 && (int32_t)t.row0 < ms[t.inst].np, "first row");
                    for (uint32_t r = t.row0; r < std::min<uint32_t>(t.row0 + c.R, ms[t.inst].np); ++r) {
                        rows[t.inst][r]++;
                        fe[t.inst][r]++;
                    }
                }
            }
        }
        for (int i = 0; i < n; ++i) {
            CHECK(where[i] != -1, "member %d in no launch", i);
            if (where[i] != 100 && where[i] != 200 && where[i] != kClasses - 1 &&
                where[i] != kClasses - 2)
                CHECK(where[i] == class_of(ms[i].nchunk), "member %d in class %d, nchunk %d", i,
                      where[i], ms[i].nchunk);
            for (int r = 0; r < ms[i].np; ++r) {
                CHECK(rows[i][r] == 1, "member %d row %d covered %d times", i, r, rows[i][r]);
                CHECK(fe[i][r] == 1, "member %d row %d closed %d times", i, r, fe[i][r]);
            }
            for (size_t q = 0; q < segs[i].size(); ++q)
                CHECK(segs[i][q] == 1, "member %d segment %zu covered %d times", i, q, segs[i][q]);
        }
    }
    CHECK(g_tuned_called, "tuned hook never consulted");
    // a member whose arena cannot hold its segment sums is refused
    std::vector<MemberShape> bad(1);
    ArenaLayout L;
    arena_layout(200000, 4096, &L);
    bad[0].np = 4096;
    bad[0].pitch = L.pitch;
    bad[0].nchunk = L.nchunk;
    bad[0].part_nseg = L.part_nseg / 2;
    PlanOptions opt;
    BatchPlan plan;
    CHECK(plan_batch(bad, opt, &plan) == QIEO_EINVAL, "short partial-sum array accepted");
}

// ---------------------------------------------------------------------------
// Snapshot headers
// ---------------------------------------------------------------------------
static void check_snapshots()
{
    const int32_t ng = 1000, np = 33;
    ArenaLayout L;
    arena_layout(ng, np, &L);
    const SnapshotId id{4u, ng, np, 777, 42ull, 0x1234ull};
    std::vector<char> buf(sizeof(StateHeader) + L.total, 0);
    auto make = [&](int64_t t, int32_t window, uint32_t elite_row) {
        std::fill(buf.begin(), buf.end(), 0);
        const StateHeader hd = make_state_header(id, t, L.total);
        std::memcpy(buf.data(), &hd, sizeof hd);
        char* body = buf.data() + sizeof hd;
        std::memcpy(body + L.tbase, &t, sizeof t);
        std::memcpy(body + L.conv + 12, &window, sizeof window);
        if (t > 0) {
            const uint64_t key = ((uint64_t)0x80000000u << 32) | (uint32_t)~elite_row;
            std::memcpy(body + L.ekey + (size_t)((t - 1) % 3) * 8, &key, 8);
        }
    };
    int64_t t = -1;
    int32_t w = -1;
    make(7, 5, 3);
    CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_OK && t == 7 && w == 5,
          "valid snapshot refused: %s", last_error());
    make(0, 0, 0);
    CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_OK && t == 0,
          "generation-0 snapshot refused");
    make(7, 5, 3);
    CHECK(check_snapshot(buf.data(), buf.size() - 1, id, L, &t, &w) == QIEO_EINVAL, "short buffer");
    CHECK(check_snapshot(buf.data(), sizeof(StateHeader) - 1, id, L, &t, &w) == QIEO_EINVAL,
          "header only");
    CHECK(check_snapshot(nullptr, buf.size(), id, L, &t, &w) == QIEO_EINVAL, "NULL buffer");
    auto refused_with = [&](SnapshotId other, const char* what) {
        CHECK(check_snapshot(buf.data(), buf.size(), other, L, &t, &w) == QIEO_EINVAL,
              "%s accepted", what);
    };
    SnapshotId o = id;
    o.elem_bytes = 8;
    refused_with(o, "other precision");
    o = id; o.n_items = ng + 1; refused_with(o, "other n_items");
    o = id; o.n_pop = np - 1; refused_with(o, "other n_pop");
    o = id; o.capacity = 778; refused_with(o, "other capacity");
    o = id; o.seed = 43; refused_with(o, "other seed");
    o = id; o.items_hash ^= 1; refused_with(o, "other items");
    // corrupted fields, one at a time
    auto corrupt = [&](size_t off, const char* what) {
        make(7, 5, 3);
        buf[off] ^= 0x5a;
        CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_EINVAL,
              "corrupted %s accepted", what);
    };
    corrupt(0, "magic");
    corrupt(offsetof(StateHeader, version), "version");
    corrupt(offsetof(StateHeader, generations), "header generations");
    corrupt(offsetof(StateHeader, arena_bytes), "arena size");
    corrupt(sizeof(StateHeader) + L.tbase, "image generation counter");
    make(7, kConvRing + 1, 3);
    CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_EINVAL, "window");
    make(7, -1, 3);
    CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_EINVAL, "negative window");
    make(7, 5, np);
    CHECK(check_snapshot(buf.data(), buf.size(), id, L, &t, &w) == QIEO_EINVAL, "elite row");
}

// ---------------------------------------------------------------------------
// Argument validation and work-shape rules
// ---------------------------------------------------------------------------
static void check_validation()
{
    CHECK(validate_shape(0, 1) == QIEO_EINVAL && validate_shape(1, 0) == QIEO_EINVAL, "zero sizes");
    CHECK(validate_shape((1 << 30) - 256, 1) == QIEO_OK, "longest row");
    CHECK(validate_shape((1 << 30) - 255, 1) == QIEO_EINVAL, "row too long");
    CHECK(validate_shape(64, 1 << 30) == QIEO_OK, "2^36 genes");
    CHECK(validate_shape(65, 1 << 30) == QIEO_EINVAL, "past 2^36 genes");
    std::vector<qieo_item> it(3, qieo_item{1, 1});
    CHECK(validate_problem(nullptr, 3, 1, 1) == QIEO_EINVAL, "NULL items");
    CHECK(validate_problem(it.data(), 3, -1, 1) == QIEO_EINVAL, "negative capacity");
    it[1].weight = -1;
    CHECK(validate_problem(it.data(), 3, 1, 1) == QIEO_EINVAL, "negative weight");
    it[1] = qieo_item{INT32_MAX - 2, 1};
    CHECK(validate_problem(it.data(), 3, 1, 1) == QIEO_OK, "profit sum INT32_MAX");
    it[1].profit += 1;
    CHECK(validate_problem(it.data(), 3, 1, 1) == QIEO_EOVERFLOW, "profit sum overflow");
    it[1] = qieo_item{1, INT32_MAX - 1};
    CHECK(validate_problem(it.data(), 3, 1, 1) == QIEO_EOVERFLOW, "weight sum overflow");
    // items hash: order and content sensitive
    std::vector<qieo_item> a = {{1, 2}, {3, 4}}, b = {{3, 4}, {1, 2}};
    CHECK(items_fnv1a(a.data(), 2) != items_fnv1a(b.data(), 2), "hash ignores order");
    CHECK(items_fnv1a(a.data(), 2) == items_fnv1a(a.data(), 2), "hash not deterministic");
    // work shapes: S never above the chunks of a row, segment order only for
    // streaming binary32 populations, cache hints only when streaming
    for (int32_t np : {1, 16, 1024, 4096, 32768})
        for (int32_t nchunk : {1, 2, 5, 40, 782}) {
            for (int elem : {4, 8}) {
                int R, S, F;
                pick_tile(np, nchunk, &R, &S, &F, elem);
                const int64_t planes = (int64_t)np * nchunk * kChunk * 2 * elem;
                CHECK(R == 1 || R == 2 || R == 4, "R");
                CHECK(S >= 1 && S <= 16 && (S <= nchunk || S == 16), "S %d for %d chunks", S, nchunk);
                CHECK(((F & kFlagSegments) != 0) == (elem == 4 && planes > (256ll << 20)),
                      "segment order rule");
                if (planes <= (256ll << 20))
                    CHECK((F & (kFlagNontemporal | kFlagNontemporalLoads)) == 0, "cache hints");
            }
        }
    for (int32_t nchunk : {1, 2, 3, 4, 7, 8, 31, 32, 1000}) {
        const int c = class_of(nchunk);
        CHECK(c >= 0 && c < kClasses && kClassWaves[c] <= std::max(nchunk, 1) * 2, "class");
    }
}

// ---------------------------------------------------------------------------
// On-chip loop planning: rows per workgroup, items per wave, LDS
// ---------------------------------------------------------------------------
static void check_onchip_plan()
{
    const size_t lim = 160 * 1024 - 256;
    OnchipPlan p;
    // 1024 x 10,000 on 256 CUs: 4 rows of 40 chunks per workgroup, 10 items a wave
    CHECK(onchip_plan(1024, 40, 256, lim, &p), "medium workload");
    CHECK(p.R == 4 && p.blocks == 256 && p.K == 10 && p.lds == onchip_lds_bytes(4, 40),
          "R %d blocks %d K %d", p.R, p.blocks, p.K);
    // every accepted shape: whole rows per workgroup, the grid covers the rows
    // once, every workgroup's items fit its waves, a compiled K, LDS in bounds
    for (int32_t np = 1; np <= 5000; np += 37) {
        for (int32_t nchunk = 1; nchunk <= 200; nchunk += 7) {
            OnchipPlan q;
            if (!onchip_plan(np, nchunk, 256, lim, &q)) {
                const int64_t R = (np + 255) / 256;
                CHECK((R * nchunk + kOnchipWaves - 1) / kOnchipWaves > kOnchipK[kOnchipVariants - 1] ||
                          onchip_lds_bytes((int)R, nchunk) > lim,
                      "%d x %d refused without cause", np, nchunk);
                continue;
            }
            CHECK(q.blocks >= 1 && q.blocks <= 256 && (int64_t)q.blocks * q.R >= np &&
                      (int64_t)(q.blocks - 1) * q.R < np,
                  "%d x %d: %d blocks of %d rows", np, nchunk, q.blocks, q.R);
            CHECK((int64_t)q.R * nchunk <= (int64_t)kOnchipWaves * q.K, "items per wave");
            bool compiled = false;
            for (int k : kOnchipK) compiled = compiled || k == q.K;
            CHECK(compiled, "K %d", q.K);
            CHECK(q.lds <= lim && q.lds % 16 == 0 &&
                      q.lds >= (2 * (size_t)nchunk * kChunk + 2 * (size_t)q.R * nchunk * 8) * 4,
                  "lds %zu", q.lds);
        }
    }
    // beyond the register budget or the LDS: refused
    CHECK(!onchip_plan(4096, 20, 256, lim, &p), "16 rows x 20 chunks per CU");
    CHECK(!onchip_plan(50, 79, 256, lim, &p), "item tables of 79 chunks exceed LDS");
    // packed item tables (one word per item) make room for them
    CHECK(onchip_plan(50, 79, 256, lim, &p, true) && p.packed && p.K == 6 &&
              p.lds == onchip_lds_bytes(1, 79, true) && p.lds < onchip_lds_bytes(1, 79) / 2 + 8192,
          "50 x 79, packed");
    CHECK(onchip_plan(50, 47, 256, lim, &p) && p.blocks == 50 && p.K == 4, "50 x 47");
    CHECK(!onchip_plan(1024, 40, 0, lim, &p) && !onchip_plan(1024, 40, 256, 0, &p),
          "no device support");
    // the default mode's choice: many rows, enough items, or long rows
    CHECK(onchip_worth(1024, 40) && onchip_worth(128, 32) && onchip_worth(24, 20) &&
              onchip_worth(4096, 4) && onchip_worth(256, 1) && onchip_worth(64, 16) &&
              onchip_worth(128, 8) && !onchip_worth(128, 4) && !onchip_worth(96, 6) &&
              !onchip_worth(255, 4) && !onchip_worth(16, 1) && !onchip_worth(64, 15),
          "onchip_worth");
}

// The batched on-chip planner's choices on hand-built members (the sizes
// worked out by hand from its rule): A = 256 rows of 70 chunks takes
// K = 10 (2 rows a workgroup, 128 workgroups, 154,624 B of LDS: 128 x 17
// us against 256 x 14.8 at K = 8); C = 256 rows of 7 chunks K = 10 (22
// rows, 12 workgroups: 12 x 17 against 15 x 14.8 at K = 8); B = 32 rows of
// 1 chunk K = 2 (one workgroup), whose launch is then emptied into a
// K = 10 launch with room.  Rows of 77 or more chunks need more than the
// 160 KB of LDS (item tables alone 2 KB a chunk) and are left out.
static void check_onchip_choices()
{
    std::vector<MemberShape> ms(3);
    const int32_t np[3] = {256, 32, 256}, nchunk[3] = {70, 1, 7};
    for (int i = 0; i < 3; ++i) {
        ms[i].np = np[i];
        ms[i].nchunk = nchunk[i];
        ms[i].pitch = nchunk[i] * kChunk;
    }
    PlanOptions opt;
    opt.onchip_blocks = 256;
    opt.onchip_lds_limit = 160 * 1024 - 256;
    opt.onchip_variants = 0x1fu;
    std::vector<OnchipLaunch> L;
    std::vector<size_t> rest;
    plan_onchip(ms, {0, 1, 2}, opt, &L, &rest);
    CHECK(rest.empty() && L.size() == 1 && L[0].K == 10 && L[0].tiles.size() == 141,
          "one K = 10 launch of 141 workgroups (got %zu launches, %zu left)", L.size(),
          rest.size());
    std::map<uint32_t, std::pair<int, int>> shape;    // member -> (R, nb)
    for (const OnchipTile& t : L[0].tiles) shape[t.inst] = {t.R, t.nb};
    CHECK(shape[0] == std::make_pair(2, 128) && shape[1] == std::make_pair(32, 1) &&
              shape[2] == std::make_pair(22, 12),
          "rows per workgroup and workgroups per member");
    // 130 workgroups a launch: A alone, C in a second K = 10 launch, B's
    // K = 2 launch emptied into A's (128 + 1 <= 130)
    opt.onchip_blocks = 130;
    plan_onchip(ms, {0, 1, 2}, opt, &L, &rest);
    CHECK(rest.empty() && L.size() == 2 && L[0].K == 10 && L[1].K == 10,
          "two K = 10 launches (got %zu)", L.size());
    size_t sizes[2] = {L[0].tiles.size(), L[1].tiles.size()};
    std::sort(sizes, sizes + 2);
    CHECK(sizes[0] == 12 && sizes[1] == 129, "launches of 12 and 129 workgroups (%zu, %zu)",
          sizes[0], sizes[1]);
    // K = 2 alone: A's rows do not fit a workgroup of 32 items, C takes one
    // row of 7 chunks ... 4 rows (28 items) a workgroup
    opt.onchip_blocks = 256;
    opt.onchip_variants = 0x01u;
    plan_onchip(ms, {0, 1, 2}, opt, &L, &rest);
    CHECK(rest.size() == 1 && rest[0] == 0, "the 70-chunk member left out at K = 2");
    // a row of 77 chunks fits no workgroup's LDS
    opt.onchip_variants = 0x1fu;
    std::vector<MemberShape> wide(1);
    wide[0].np = 8;
    wide[0].nchunk = 77;
    wide[0].pitch = 77 * kChunk;
    plan_onchip(wide, {0}, opt, &L, &rest);
    CHECK(L.empty() && rest.size() == 1, "a 77-chunk row placed");
    wide[0].nchunk = 76;
    wide[0].pitch = 76 * kChunk;
    plan_onchip(wide, {0}, opt, &L, &rest);
    CHECK(L.size() == 1 && rest.empty(), "a 76-chunk row left out");
    // packed item tables (1 KB a chunk, with 12 words a chunk of allele
    // words at one row per workgroup): rows of up to 146 chunks fit
    wide[0].packed = true;
    for (int nc : {77, 146}) {
        wide[0].nchunk = nc;
        wide[0].pitch = nc * kChunk;
        plan_onchip(wide, {0}, opt, &L, &rest);
        CHECK(L.size() == 1 && rest.empty() && L[0].packed, "a packed %d-chunk row left out", nc);
    }
    wide[0].nchunk = 147;
    wide[0].pitch = 147 * kChunk;
    plan_onchip(wide, {0}, opt, &L, &rest);
    CHECK(L.empty() && rest.size() == 1, "a packed 147-chunk row placed");
    // items_packable: both halves within [0, 2^14 - 1]
    {
        qieo_item it[2] = {{kPackedItemMax, kPackedItemMax}, {0, 1}};
        CHECK(items_packable(it, 2), "items at the packed maximum refused");
        it[1].profit = kPackedItemMax + 1;
        CHECK(!items_packable(it, 2), "a profit of 2^14 accepted");
        it[1].profit = 5;
        it[1].weight = kPackedItemMax + 1;
        CHECK(!items_packable(it, 2), "a weight of 2^14 accepted");
    }
    // windows apart: B with a window goes to a launch of its own
    opt.onchip_variants = 0x1fu;
    ms[1].conv = true;
    plan_onchip(ms, {0, 1, 2}, opt, &L, &rest);
    CHECK(L.size() == 2, "a window-testing launch apart (%zu launches)", L.size());
    for (const OnchipLaunch& x : L)
        for (const OnchipTile& t : x.tiles) CHECK(ms[t.inst].conv == x.conv, "window test mixed");
}

int main()
{
    check_arena();
    check_historical_overflow();
    check_seg_map();
    check_offset_allocator();
    check_plan_batch();
    check_snapshots();
    check_validation();
    check_onchip_plan();
    check_onchip_choices();
    std::printf("host checks passed: %d\n", g_checks);
    return 0;
}
