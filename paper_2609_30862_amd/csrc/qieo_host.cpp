// Host-side planning of the library (see qieo_host.hpp).  No HIP calls.
#include "qieo_host.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

namespace qieo {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// Arena
// ---------------------------------------------------------------------------
static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t arena_layout(int32_t ng, int32_t np, ArenaLayout* L, int elem)
{
    const int32_t pitch = (int32_t)align_up((size_t)ng, 64);
    const int32_t nchunk = (pitch + kChunk - 1) / kChunk;
    const size_t wpr = (size_t)nchunk * kWordsPerChunk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L->pitch = pitch;
    L->nchunk = nchunk;
    L->alpha = take(((size_t)np * pitch + kChunk) * (size_t)elem);
    L->beta = take(((size_t)np * pitch + kChunk) * (size_t)elem);
    L->xbits = take(2 * (size_t)np * wpr * sizeof(uint32_t));
    L->v = take((size_t)nchunk * kChunk * sizeof(int32_t));
    L->w = take((size_t)nchunk * kChunk * sizeof(int32_t));
    L->fit = take(2 * (size_t)np * sizeof(int32_t));
    L->prof = take(2 * (size_t)np * sizeof(int32_t));
    L->wt = take(2 * (size_t)np * sizeof(int32_t));
    L->ekey = take(3 * sizeof(unsigned long long));
    L->best = take(8 * sizeof(int32_t));
    L->best_bits = take(wpr * sizeof(uint32_t));
    L->tbase = take(sizeof(int64_t));
    L->conv = take(64 * sizeof(int32_t));
    L->sync = take(16 * sizeof(uint32_t) +
                   2 * (size_t)std::min(np, (int32_t)kOnchipMaxBlocks) * sizeof(uint64_t));
    // the segment sums: the last block, so a launch with shorter segments
    // than this sizing would write past the arena's end (segments_fit)
    L->part_nseg = (int32_t)seg_count(nchunk, kSegChunksMin);
    L->part = take((size_t)L->part_nseg * (size_t)np * 2 * sizeof(uint32_t));
    L->total = off;
    // everything except the amplitude planes themselves is zero-initialised
    L->zero_from = 0;
    return off;
}

bool segments_fit(const ArenaLayout& L, int sc)
{
    return sc >= 1 && seg_count(L.nchunk, sc) <= (int64_t)L.part_nseg;
}

int validate_shape(int32_t n_items, int32_t n_pop)
{
    if (n_items < 1) return set_error(QIEO_EINVAL, "n_items must be >= 1 (got %d)", n_items);
    if (n_pop < 1) return set_error(QIEO_EINVAL, "n_pop must be >= 1 (got %d)", n_pop);
    if (n_items > (1 << 30) - 256)
        return set_error(QIEO_EINVAL, "n_items too large (%d)", n_items);
    // keeps every plane size in the arena layout far from size_t wrap-around
    // (2^36 genes is 512 GB of binary32 amplitudes, beyond any one device)
    if ((int64_t)n_pop * (int64_t)align_up((size_t)n_items, 64) > ((int64_t)1 << 36))
        return set_error(QIEO_EINVAL, "population of %d x %d genes exceeds 2^36 genes", n_pop,
                         n_items);
    return QIEO_OK;
}

int validate_problem(const qieo_item* items, int32_t n_items, int32_t capacity, int32_t n_pop)
{
    if (!items) return set_error(QIEO_EINVAL, "items is NULL");
    int rc = validate_shape(n_items, n_pop);
    if (rc) return rc;
    if (capacity < 0) return set_error(QIEO_EINVAL, "capacity must be >= 0 (got %d)", capacity);
    int64_t sv = 0, sw = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        if (items[i].profit < 0 || items[i].weight < 0)
            return set_error(QIEO_EINVAL, "item %d has a negative profit or weight", i);
        sv += items[i].profit;
        sw += items[i].weight;
    }
    if (sv > INT32_MAX || sw > INT32_MAX)
        return set_error(QIEO_EOVERFLOW,
                         "sum of profits (%lld) or weights (%lld) exceeds INT32_MAX",
                         (long long)sv, (long long)sw);
    return QIEO_OK;
}

uint64_t items_fnv1a(const qieo_item* items, int32_t n)
{
    uint64_t x = 0xcbf29ce484222325ull;
    const unsigned char* p = reinterpret_cast<const unsigned char*>(items);
    for (size_t k = 0; k < (size_t)n * sizeof(qieo_item); ++k) {
        x ^= p[k];
        x *= 0x100000001b3ull;
    }
    return x;
}

// ---------------------------------------------------------------------------
// Work shapes
// ---------------------------------------------------------------------------

// Variant bits for a work shape, from sweeps over fifteen (Np, Ng) shapes
// between 82 MB and 13 GB of amplitudes.  Once the planes one generation
// streams exceed the 256 MB last-level cache: non-temporal loads (cached
// amplitudes would only evict the item tables and allele words) and
// non-temporal stores (nothing written survives until the next generation
// reads it).  Below that size both hints cost time (up to 27 %): the next
// generation's reads may still hit the cache.  Prefetch when a wave walks
// more than one chunk, except in multi-row workgroups over long rows (>= 32
// chunks per wave), where several rows' loads already keep enough in flight
// and the prefetch buffers cost occupancy.
int variant_flags(int R, int S, int64_t nchunk, int64_t plane_bytes)
{
    int f = 0;
    if (plane_bytes > ((int64_t)256 << 20)) f |= kFlagNontemporal | kFlagNontemporalLoads;
    if (nchunk > S && !(R >= 2 && nchunk >= 32 * (int64_t)S)) f |= kFlagPrefetch;
    return f;
}

// Work shape for a single instance: rows per workgroup R, waves per
// workgroup S and kernel variant flags.  Whole rows stay in one workgroup
// (Evaluation closes in LDS); S splits the gene axis.  R is the largest of
// 4, 2, 1 that still leaves >= 32 wavefronts per CU (8192 on 256 CUs), since
// more rows per workgroup amortise the item-table and elite-mask reads.
// Streaming populations (planes beyond the last-level cache) with long rows
// (>= 32 chunks) and at least 1024 of them take 2 rows x 16 waves, the
// fastest row shape on every such workload measured.  Streaming binary32
// populations run in segment order instead: faster than the best row shape
// on all ten streaming workloads measured (6-14 %; 2.23 ms against 2.56 on
// 4096 x 200,000), slower on cache-resident ones (11-18 %), where the row
// kernel stays.
void pick_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags, int elem_bytes)
{
    const int64_t plane_bytes = (int64_t)np * nchunk * kChunk * 2 * (int64_t)elem_bytes;
    int s = 8;
    if (nchunk < s) s = std::max(1, nchunk);
    int r = 1;
    for (int cand : {4, 2}) {
        if ((int64_t)((np + cand - 1) / cand) * s >= 8192) { r = cand; break; }
    }
    if (plane_bytes > ((int64_t)256 << 20) && nchunk >= 32 && np >= 1024) {
        r = 2;
        s = 16;
    }
    *R = r;
    *S = s;
    *flags = variant_flags(r, s, nchunk, plane_bytes);
    if (elem_bytes == 4 && plane_bytes > ((int64_t)256 << 20))
        *flags = kFlagSegments | kFlagNontemporal | kFlagNontemporalLoads;
}

size_t resident_lds_bytes(int32_t np, int32_t pitch, int32_t nchunk)
{
    const size_t wpr = (size_t)nchunk * kWordsPerChunk;
    const size_t words = 2 * (size_t)np * pitch + 2 * (size_t)np * wpr + wpr +
                         2 * (size_t)nchunk * kChunk + 10 * (size_t)np;
    return words * sizeof(uint32_t);
}

size_t onchip_lds_bytes(int R, int32_t nchunk, bool packed)
{
    const size_t wpr = (size_t)nchunk * kWordsPerChunk;
    const size_t words = (packed ? 1 : 2) * (size_t)nchunk * kChunk + 2 * (size_t)R * wpr + wpr +
                         8 * (size_t)R;
    return (words * sizeof(uint32_t) + 15) / 16 * 16;
}

bool items_packable(const qieo_item* items, int32_t n)
{
    for (int32_t i = 0; i < n; ++i)
        if (items[i].profit < 0 || items[i].profit > kPackedItemMax || items[i].weight < 0 ||
            items[i].weight > kPackedItemMax)
            return false;
    return true;
}

bool onchip_worth(int32_t np, int32_t nchunk)
{
    return np >= 256 || (int64_t)np * nchunk >= 1024 || nchunk >= 20;
}

bool onchip_plan(int32_t np, int32_t nchunk, int n_cu, size_t lds_limit, OnchipPlan* out,
                 bool packed)
{
    // rows travel in 16 bits of the workgroups' keys
    if (np < 1 || np > 65536 || nchunk < 1 || n_cu < 1 || n_cu > kOnchipMaxBlocks) return false;
    const int64_t R = (np + (int64_t)n_cu - 1) / n_cu;
    const int64_t need = (R * nchunk + kOnchipWaves - 1) / kOnchipWaves;
    int K = 0;
    for (int k : kOnchipK)
        if (k >= need) { K = k; break; }
    if (K == 0) return false;
    const size_t lds = onchip_lds_bytes((int)R, nchunk, packed);
    if (lds > lds_limit) return false;
    out->packed = packed;
    out->R = (int)R;
    out->blocks = (int)((np + R - 1) / R);
    out->K = K;
    out->lds = lds;
    return true;
}

SegMap seg_map_for(int64_t n_seg, int xcds, int32_t nseg_row)
{
    SegMap m{};
    m.xcds = xcds < 1 ? 1 : xcds;
    m.xshift = -1;
    for (int b = 0; b < 31; ++b)
        if (m.xcds == (1 << b)) m.xshift = b;
    m.q = (int32_t)(n_seg / m.xcds);
    m.r = (int32_t)(n_seg % m.xcds);
    if (nseg_row > 0) {
        // (s * magic) >> mshift equals s / nseg for every s < 2^31 with
        // mshift = 31 + ceil(log2 nseg), magic = ceil(2^mshift / nseg): the
        // rounding error of magic, below 1, times s < 2^31 stays under
        // 2^mshift / nseg, too little to reach the next multiple.
        int l = 0;
        while ((1ll << l) < nseg_row) ++l;
        m.nseg = nseg_row;
        m.mshift = 31 + l;
        m.magic = (uint64_t)((((unsigned __int128)1 << m.mshift) + (unsigned)nseg_row - 1) /
                             (unsigned)nseg_row);
    }
    return m;
}

// ---------------------------------------------------------------------------
// Offset allocator
// ---------------------------------------------------------------------------
static size_t round256(size_t x) { return (x + 255) / 256 * 256; }

void OffsetAllocator::reset(size_t capacity)
{
    cap_ = round256(std::max<size_t>(capacity, 256));
    used_ = 0;
    free_.clear();
    busy_.clear();
    free_[0] = cap_;
}

size_t OffsetAllocator::alloc(size_t bytes)
{
    if (bytes > cap_) return npos;
    bytes = round256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        busy_[off] = bytes;
        used_ += bytes;
        return off;
    }
    return npos;
}

bool OffsetAllocator::release(size_t off)
{
    auto b = busy_.find(off);
    if (b == busy_.end()) return false;
    size_t start = off, sz = b->second;
    busy_.erase(b);
    used_ -= sz;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + sz == next->first) {
        sz += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == start) {
            start = prev->first;
            sz += prev->second;
            free_.erase(prev);
        }
    }
    free_[start] = sz;
    return true;
}

size_t OffsetAllocator::largest_free() const
{
    size_t m = 0;
    for (auto& f : free_) m = std::max(m, f.second);
    return m;
}

bool OffsetAllocator::check() const
{
    // every byte of [0, cap) in exactly one block; free blocks never adjacent
    std::map<size_t, std::pair<size_t, bool>> all;
    for (auto& f : free_) all[f.first] = {f.second, true};
    for (auto& b : busy_) {
        if (all.count(b.first)) return false;
        all[b.first] = {b.second, false};
    }
    size_t pos = 0, used = 0;
    bool prev_free = false;
    for (auto& a : all) {
        if (a.first != pos || a.second.first == 0 || a.first % 256 || a.second.first % 256)
            return false;
        if (a.second.second && prev_free) return false;
        prev_free = a.second.second;
        if (!a.second.second) used += a.second.first;
        pos += a.second.first;
    }
    return pos == cap_ && used == used_;
}

// ---------------------------------------------------------------------------
// Batch shape classes and tile tables
// ---------------------------------------------------------------------------
int class_of(int32_t nchunk)
{
    if (nchunk <= 1) return 0;
    if (nchunk <= 3) return 1;
    if (nchunk <= 7) return 2;
    if (nchunk <= 31) return 3;
    return 4;
}

namespace {

struct OnchipPlace {
    size_t id;
    int32_t R, nb;
    size_t lds;
};

// Member m on workgroups of variant v: false if it does not fit.
bool onchip_fit(const MemberShape& m, size_t id, int v, const PlanOptions& opt, OnchipPlace* out)
{
    const int K = kOnchipK[v];
    const int64_t cap = (int64_t)kOnchipWaves * K;          // items a workgroup holds
    if (m.np < 1 || m.np > 65536 || m.nchunk < 1 || m.nchunk > cap) return false;
    int64_t R = std::min<int64_t>(m.np, cap / m.nchunk);
    int64_t nb = (m.np + R - 1) / R;
    R = (m.np + nb - 1) / nb;                               // balanced: same nb, fewer rows
    nb = (m.np + R - 1) / R;
    const size_t lds = onchip_lds_bytes((int)R, m.nchunk, m.packed);
    if (nb > opt.onchip_blocks || lds > opt.onchip_lds_limit) return false;
    *out = OnchipPlace{id, (int32_t)R, (int32_t)nb, lds};
    return true;
}

// Measured cost of one generation of a launch of variant v, in us.
double onchip_launch_cost(int v) { return 6.0 + 1.1 * kOnchipK[v]; }

}  // namespace

void plan_onchip(const std::vector<MemberShape>& members, const std::vector<size_t>& ids,
                 const PlanOptions& opt, std::vector<OnchipLaunch>* out, std::vector<size_t>* rest)
{
    out->clear();
    rest->clear();
    // [variant][has a window][packed item tables]
    std::vector<std::vector<OnchipPlace>> by_variant(4 * kOnchipVariants);
    for (size_t i : ids) {
        const MemberShape& m = members[i];
        int best = -1;
        double best_cost = 0.0;
        OnchipPlace pick{};
        for (int v = 0; v < kOnchipVariants && opt.onchip_blocks > 0; ++v) {
            if (!(opt.onchip_variants & (1u << v))) continue;
            OnchipPlace q;
            if (!onchip_fit(m, i, v, opt, &q)) continue;
            // the member's share of a launch's generation: its workgroups
            // times the cost of one workgroup-generation of variant K
            const double cost = (double)q.nb * onchip_launch_cost(v);
            if (best < 0 || cost < best_cost) {
                best = v;
                best_cost = cost;
                pick = q;
            }
        }
        if (best < 0) rest->push_back(i);
        else by_variant[4 * best + (m.conv ? 2 : 0) + (m.packed ? 1 : 0)].push_back(pick);
    }
    // per variant and window test, first fit by decreasing workgroup count
    struct Bin {
        int v;
        bool conv, packed;
        int64_t used;
        std::vector<OnchipPlace> items;
    };
    std::vector<Bin> bins;
    for (int vc = 4 * kOnchipVariants - 1; vc >= 0; --vc) {
        std::vector<OnchipPlace>& placed = by_variant[vc];
        if (placed.empty()) continue;
        std::stable_sort(placed.begin(), placed.end(),
                         [](const OnchipPlace& a, const OnchipPlace& b) { return a.nb > b.nb; });
        const size_t first = bins.size();
        for (const OnchipPlace& q : placed) {
            size_t b = first;
            while (b < bins.size() && bins[b].used + q.nb > opt.onchip_blocks) ++b;
            if (b == bins.size()) bins.push_back(Bin{vc / 4, (vc & 2) != 0, (vc & 1) != 0, 0, {}});
            bins[b].used += q.nb;
            bins[b].items.push_back(q);
        }
    }
    // A launch costs the same per generation however few of its workgroups
    // are used, so a launch whose members all fit the spare workgroups of
    // launches of a larger variant (same window test) is emptied into them:
    // cheapest launches first, each member first-fit into the largest
    // variants first, all or nothing.
    std::vector<size_t> order(bins.size());
    for (size_t b = 0; b < bins.size(); ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return bins[a].v < bins[b].v; });
    std::vector<bool> gone(bins.size(), false);
    for (size_t src : order) {
        std::vector<int64_t> used(bins.size());
        for (size_t b = 0; b < bins.size(); ++b) used[b] = bins[b].used;
        std::vector<std::pair<size_t, OnchipPlace>> moves;
        bool all = true;
        for (const OnchipPlace& q : bins[src].items) {
            bool placed = false;
            for (size_t dst = 0; dst < bins.size() && !placed; ++dst) {
                if (gone[dst] || dst == src || bins[dst].conv != bins[src].conv ||
                    bins[dst].packed != bins[src].packed || bins[dst].v <= bins[src].v)
                    continue;
                OnchipPlace r;
                if (onchip_fit(members[q.id], q.id, bins[dst].v, opt, &r) &&
                    used[dst] + r.nb <= opt.onchip_blocks) {
                    used[dst] += r.nb;
                    moves.emplace_back(dst, r);
                    placed = true;
                }
            }
            if (!placed) {
                all = false;
                break;
            }
        }
        if (!all) continue;
        for (auto& mv : moves) {
            bins[mv.first].used += mv.second.nb;
            bins[mv.first].items.push_back(mv.second);
        }
        bins[src].items.clear();
        bins[src].used = 0;
        gone[src] = true;
    }
    for (size_t b = 0; b < bins.size(); ++b) {
        if (gone[b]) continue;
        Bin& bin = bins[b];
        OnchipLaunch L;
        L.K = kOnchipK[bin.v];
        L.conv = bin.conv;
        L.packed = bin.packed;
        // members in index order inside a launch
        std::sort(bin.items.begin(), bin.items.end(),
                  [](const OnchipPlace& a, const OnchipPlace& c) { return a.id < c.id; });
        for (const OnchipPlace& q : bin.items) {
            const int32_t np = members[q.id].np;
            for (int32_t w = 0; w < q.nb; ++w) {
                OnchipTile t{};
                t.inst = (uint32_t)q.id;
                t.row0 = w * q.R;
                t.nrows = std::min(q.R, np - t.row0);
                t.R = q.R;
                t.blk = w;
                t.nb = q.nb;
                L.tiles.push_back(t);
            }
            L.lds = std::max(L.lds, q.lds);
        }
        out->push_back(std::move(L));
    }
}

int plan_batch(const std::vector<MemberShape>& members, const PlanOptions& opt, BatchPlan* out)
{
    out->resident.clear();
    out->resident_lds = 0;
    out->onchip.clear();
    out->classes.clear();
    const size_t n = members.size();
    if (n > (size_t)UINT32_MAX) return set_error(QIEO_EINVAL, "too many members (%zu)", n);

    // The batched on-chip loop takes every member it can place (not under a
    // forced shape): its workgroups hold their members' planes in registers
    // for the whole call, at about 6e11 gene-updates/s for the chip (vector
    // ALU bound) against about 3.7e11 streamed from HBM at 16 B a gene.
    std::vector<size_t> rest;
    {
        std::vector<size_t> all(n);
        for (size_t i = 0; i < n; ++i) all[i] = i;
        if (opt.onchip_blocks > 0 && opt.force_R == 0)
            plan_onchip(members, all, opt, &out->onchip, &rest);
        else
            rest = std::move(all);
    }
    // of the others, members whose whole state fits in one workgroup's LDS
    // run the call there (one workgroup each); the rest are grouped by shape
    // class
    std::vector<std::vector<size_t>> groups(kClasses);
    for (size_t i : rest) {
        const MemberShape& m = members[i];
        const size_t lds = resident_lds_bytes(m.np, m.pitch, m.nchunk);
        if (opt.use_persistent && lds <= opt.lds_limit) {
            out->resident.push_back((uint32_t)i);
            out->resident_lds = std::max(out->resident_lds, lds);
        } else {
            groups[class_of(m.nchunk)].push_back(i);
        }
    }
    // largest first: the longest workgroups start first
    std::stable_sort(out->resident.begin(), out->resident.end(), [&](uint32_t a, uint32_t b) {
        return (int64_t)members[a].np * members[a].pitch > (int64_t)members[b].np * members[b].pitch;
    });
    // amplitude bytes one generation of the batch streams, on-chip members
    // aside (the classes run side by side, so they share the caches)
    int64_t plane_bytes = 0;
    for (size_t i : rest)
        plane_bytes += (int64_t)members[i].np * members[i].pitch * 2 * (int64_t)sizeof(float);
    // A batch that streams from HBM runs the rows of 8 or more chunks in
    // segment order, all in one table (one launch pair per generation), when
    // that table stays within kMaxSegTiles; else only the >= 32-chunk class
    // does, if its own table fits.  On the 512-instance ragged batch: 0.330 s
    // per 500 generations merged, 0.333 s with the 8-31-chunk class in row
    // order beside it (as a segment-order class of its own on a second
    // stream it measured 0.339 s; every class of the batch in the one
    // table, 0.333 s).
    auto seg_tiles_of = [&](const std::vector<size_t>& g) {
        int64_t n_tiles = 0;
        for (size_t i : g) n_tiles += (int64_t)members[i].np * seg_count(members[i].nchunk, kSegChunks32);
        return n_tiles;
    };
    const bool streaming = opt.use_segments && opt.force_R == 0 && plane_bytes > ((int64_t)256 << 20);
    if (streaming && opt.merge_segments && !groups[kClasses - 2].empty() &&
        seg_tiles_of(groups[kClasses - 2]) + seg_tiles_of(groups[kClasses - 1]) <= kMaxSegTiles) {
        auto& g4 = groups[kClasses - 1];
        g4.insert(g4.end(), groups[kClasses - 2].begin(), groups[kClasses - 2].end());
        groups[kClasses - 2].clear();
    }
    for (int c = 0; c < kClasses; ++c) {
        auto& g = groups[c];
        if (g.empty()) continue;
        std::sort(g.begin(), g.end(), [&](size_t a, size_t b) {
            if (members[a].nchunk != members[b].nchunk) return members[a].nchunk > members[b].nchunk;
            return a < b;
        });
        ClassPlan sc;
        sc.cls = c;
        for (size_t i : g) {
            sc.rows += members[i].np;
            sc.max_nchunk = std::max(sc.max_nchunk, members[i].nchunk);
        }
        sc.S = kClassWaves[c];
        sc.R = 1;
        // long rows: at most 2 rows per 16-wave workgroup, as for single
        // streaming populations
        for (int cand : {4, 2}) {
            if (sc.S == 16 && cand > 2) continue;
            // blocks of the class at R rows each, times S waves: keep >= 8192 waves
            int64_t blocks = 0;
            for (size_t i : g) blocks += (members[i].np + cand - 1) / cand;
            if (blocks * sc.S >= 8192) { sc.R = cand; break; }
        }
        sc.flags = variant_flags(sc.R, sc.S, sc.max_nchunk, plane_bytes);
        int tR = 0, tS = 0, tF = 0;
        if (opt.force_R > 0) {
            sc.R = opt.force_R;
            sc.S = opt.force_S;
            sc.flags = opt.force_flags;
        } else if (opt.tuned && opt.tuned(c, sc.rows, sc.max_nchunk, &tR, &tS, &tF)) {
            sc.R = tR;
            sc.S = tS;
            sc.flags = tF;
            sc.tuned = true;
        }
        // The long-row class of a batch that streams from HBM (rows of 8 or
        // more chunks when the classes were merged above, else of 32 or
        // more) runs in segment order: one tile per 1024-gene segment,
        // members in arena address order, so the class sweeps its planes in
        // address order; a second tile table gives the closing launch four
        // rows per workgroup.  The segment table costs 8 bytes per 1024
        // genes and is rebuilt on every membership change; a server holding
        // thousands of residents changes membership every few generations,
        // so a class of more than kMaxSegTiles segments keeps row order.  A
        // tuned shape of this class says whether segment order pays.
        bool seg = c == kClasses - 1 && streaming && seg_tiles_of(g) <= kMaxSegTiles;
        if (sc.tuned) seg = seg && (sc.flags & kFlagSegments);
        else if (seg) sc.flags = kFlagSegments | kFlagNontemporal | kFlagNontemporalLoads;
        if (!seg) sc.flags &= ~kFlagSegments;
        if (seg) {
            std::sort(g.begin(), g.end(), [&](size_t a, size_t b) {
                return members[a].addr < members[b].addr;
            });
            for (size_t i : g) {
                const MemberShape& m = members[i];
                const int64_t nseg = seg_count(m.nchunk, kSegChunks32);
                if (nseg > m.part_nseg)
                    return set_error(QIEO_EINVAL, "member %zu: %lld segments per row exceed its "
                                     "arena's %d", i, (long long)nseg, m.part_nseg);
                for (int64_t q = 0; q < (int64_t)m.np * nseg; ++q)
                    sc.tiles.push_back(Tile{(uint32_t)i, (uint32_t)q});
                for (int32_t r0 = 0; r0 < m.np; r0 += 4)
                    sc.fe_tiles.push_back(Tile{(uint32_t)i, (uint32_t)r0});
            }
        } else {
            for (size_t i : g)
                for (int32_t r0 = 0; r0 < members[i].np; r0 += sc.R)
                    sc.tiles.push_back(Tile{(uint32_t)i, (uint32_t)r0});
        }
        if (sc.tiles.size() > (size_t)INT32_MAX || sc.fe_tiles.size() > (size_t)INT32_MAX)
            return set_error(QIEO_EINVAL, "tile table too large");
        out->classes.push_back(std::move(sc));
    }
    return QIEO_OK;
}

// ---------------------------------------------------------------------------
// Snapshots
// ---------------------------------------------------------------------------
static constexpr char kStateMagic[8] = {'Q', 'I', 'E', 'O', 'S', 'T', 'A', 'T'};
static constexpr uint32_t kStateVersion = 2;

StateHeader make_state_header(const SnapshotId& id, int64_t generations, uint64_t arena_bytes)
{
    StateHeader hd{};
    std::memcpy(hd.magic, kStateMagic, sizeof hd.magic);
    hd.version = kStateVersion;
    hd.elem_bytes = id.elem_bytes;
    hd.n_items = id.n_items;
    hd.n_pop = id.n_pop;
    hd.capacity = id.capacity;
    hd.seed = id.seed;
    hd.items_hash = id.items_hash;
    hd.generations = generations;
    hd.arena_bytes = arena_bytes;
    return hd;
}

int check_snapshot(const void* buf, size_t bytes, const SnapshotId& id, const ArenaLayout& L,
                   int64_t* generations, int32_t* window)
{
    if (!buf) return set_error(QIEO_EINVAL, "NULL argument");
    if (bytes < sizeof(StateHeader)) return set_error(QIEO_EINVAL, "state buffer too short");
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, kStateMagic, sizeof hd.magic) != 0 || hd.version != kStateVersion)
        return set_error(QIEO_EINVAL, "not a libqieo state snapshot (or another version)");
    if (hd.elem_bytes != id.elem_bytes)
        return set_error(QIEO_EINVAL, "snapshot precision differs from the handle's");
    if (hd.n_items != id.n_items || hd.n_pop != id.n_pop || hd.capacity != id.capacity ||
        hd.seed != id.seed || hd.items_hash != id.items_hash)
        return set_error(QIEO_EINVAL, "snapshot belongs to another problem (items, capacity, "
                                      "population size or seed differ)");
    if (hd.arena_bytes != L.total || bytes - sizeof hd < hd.arena_bytes)
        return set_error(QIEO_EINVAL, "snapshot size does not match the handle's state");
    const char* body = (const char*)buf + sizeof hd;
    int64_t tb;
    int32_t win;
    std::memcpy(&tb, body + L.tbase, sizeof tb);
    std::memcpy(&win, body + L.conv + 3 * sizeof(int32_t), sizeof win);
    if (tb != hd.generations || tb < 0 || tb > (int64_t)INT32_MAX || win < 0 || win > kConvRing)
        return set_error(QIEO_EINVAL, "snapshot is inconsistent");
    if (tb > 0) {
        // the next generation rotates toward the elite row its key names
        // (row = ~low word): a row outside the population would be read out
        // of bounds on the device
        uint64_t key;
        std::memcpy(&key, body + L.ekey + (size_t)((tb - 1) % 3) * sizeof key, sizeof key);
        if ((uint32_t)~(uint32_t)key >= (uint32_t)id.n_pop)
            return set_error(QIEO_EINVAL, "snapshot is inconsistent (elite row out of range)");
    }
    *generations = tb;
    *window = win;
    return QIEO_OK;
}

}  // namespace qieo
