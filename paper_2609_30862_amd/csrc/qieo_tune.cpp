// Work-shape autotuner and its database.
//
// The generation kernel's speed depends on rows per workgroup R, wavefronts
// per workgroup S and the variant flags, never its results.  The tuner times
// every candidate on a scratch population of the caller's shape (its own
// arena; the caller's trajectory untouched), picks the fastest, and records
// it under the shape's bucket (log2 of rows, log2 of 256-gene chunks per
// row).  qieo_create consults the database before falling back to the
// built-in rule.  Every candidate starts from the same state (a device copy
// of the scratch arena taken after two warm-up generations) and runs the
// same generations, so each does the same work: later candidates are not
// timed on a more converged population, whose rows tied with the elite skip
// the rotation.  Candidates are timed twice, in opposite orders, and keep
// the faster time.
//
// The same database holds batch launch classes (shape class, log2 of the
// class's rows, log2 of its longest row in chunks), filled by
// qieo_batch_autotune and consulted when a batch or server engine builds
// its classes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qieo.h"
#include "qieo_internal.hpp"

namespace qieo {

namespace {

struct Entry {
    int R, S, flags;
    double ms;
};

// key: {kind, a, b, c}: kind 0 = single instance {log2 rows, log2 chunks, 0};
// kind 1 = batch class {class, log2 rows, log2 longest row in chunks}, class
// -1 = a batch's on-chip variant subset {-1, log2 of all its rows, log2 of
// its longest row} with R = launches, S = waves, flags = the subset
using Key = std::tuple<int, int, int, int>;

std::mutex g_db_mu;
std::map<Key, Entry> g_db;

int ilog2(int64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

Key instance_key(int32_t np, int32_t nchunk) { return Key{0, ilog2(np), ilog2(nchunk), 0}; }

Key class_key(int cls, int64_t rows, int32_t max_nchunk)
{
    return Key{1, cls, ilog2(rows), ilog2(max_nchunk)};
}

}  // namespace

bool tuned_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags)
{
    std::lock_guard<std::mutex> lk(g_db_mu);
    auto it = g_db.find(instance_key(np, nchunk));
    if (it == g_db.end()) return false;
    *R = it->second.R;
    *S = std::min(it->second.S, std::max(1, (int)nchunk));
    *flags = it->second.flags;
    return true;
}

bool tuned_class(int cls, int64_t rows, int32_t max_nchunk, int* R, int* S, int* flags)
{
    std::lock_guard<std::mutex> lk(g_db_mu);
    auto it = g_db.find(class_key(cls, rows, max_nchunk));
    if (it == g_db.end()) return false;
    *R = it->second.R;
    *S = it->second.S;
    *flags = it->second.flags;
    return true;
}

void record_class(int cls, int64_t rows, int32_t max_nchunk, int R, int S, int flags, double ms)
{
    std::lock_guard<std::mutex> lk(g_db_mu);
    g_db[class_key(cls, rows, max_nchunk)] = Entry{R, S, flags, ms};
}

// Items like the workloads' correlated ones: weights uniform in [1, 100]
// (a 64-bit LCG), value = weight + 10, capacity half the weight sum.
void synthetic_items(int32_t n, std::vector<qieo_item>* items, int32_t* capacity)
{
    items->resize((size_t)n);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    int64_t sum = 0;
    for (int32_t i = 0; i < n; ++i) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        const int32_t w = 1 + (int32_t)((x >> 33) % 100);
        (*items)[(size_t)i] = qieo_item{w + 10, w};
        sum += w;
    }
    *capacity = (int32_t)(sum / 2);
}

}  // namespace qieo

using namespace qieo;

extern "C" int qieo_autotune(int32_t n_items, int32_t n_pop, const qieo_item* items,
                             int32_t capacity, int32_t trial_generations,
                             qieo_tune_result* out)
{
    clear_error();
    if (trial_generations < 1 || trial_generations > 1000)
        return set_error(QIEO_EINVAL, "trial_generations must be in [1, 1000] (got %d)",
                         trial_generations);
    // before the synthetic item table below is sized by n_items
    int rc = validate_shape(n_items, n_pop);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    std::vector<qieo_item> synth;
    if (!items) {
        synthetic_items(n_items, &synth, &capacity);
        items = synth.data();
    }
    if ((rc = validate_problem(items, n_items, capacity, n_pop))) return rc;
    ArenaLayout L;
    arena_layout(n_items, n_pop, &L);
    char* arena = nullptr;
    char* backup = nullptr;
    InstDev* d_desc = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (arena) (void)hipFree(arena);
        if (backup) (void)hipFree(backup);
        if (d_desc) (void)hipFree(d_desc);
        if (s) (void)hipStreamDestroy(s);
    };
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        rc = hip_fail(e, "stream/event creation");
        cleanup();
        return rc;
    }
    if (hipMalloc((void**)&arena, L.total) != hipSuccess ||
        hipMalloc((void**)&backup, L.total) != hipSuccess ||
        hipMalloc((void**)&d_desc, sizeof(InstDev)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_error(QIEO_ENOMEM, "scratch population of 2 x %zu bytes does not fit", L.total);
    }
    InstDev d = bind_arena(arena, L, n_items, n_pop, capacity, 0x7475ull);
    std::vector<int32_t> staging;
    if ((rc = upload_and_init(d, items, s, L, arena, staging))) {
        cleanup();
        return rc;
    }
    if ((e = hipMemcpyAsync(d_desc, &d, sizeof d, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        rc = hip_fail(e, "descriptor upload");
        cleanup();
        return rc;
    }
    // candidates: R x S x flags; S never above the chunks per row
    std::vector<Entry> cand;
    for (int R : {1, 2, 4})
        for (int S : {2, 4, 8, 16}) {
            if (S > std::max(2, L.nchunk) && S != 2) continue;
            for (int f = 0; f < kFlagSegments; ++f) cand.push_back(Entry{R, S, f, 1e300});
        }
    // segment order: the work shape does not apply, only the cache hints
    for (int f : {0, kFlagNontemporal, kFlagNontemporalLoads, kFlagNontemporal | kFlagNontemporalLoads})
        cand.push_back(Entry{1, kSegWaves32, kFlagSegments | f, 1e300});
    // gens launches of candidate c from generation tbase
    auto launch = [&](const Entry& c, int gens) -> hipError_t {
        const int blocks = (n_pop + c.R - 1) / c.R;
        hipError_t ee = hipSuccess;
        for (int k = 0; k < gens && ee == hipSuccess; ++k)
            ee = (c.flags & kFlagSegments)
                     ? launch_segments(d_desc, n_pop, L.nchunk, L.part_nseg, c.flags, k, gens,
                                       false, s)
                     : launch_generation(d_desc, nullptr, blocks, c.R, c.S, c.flags, k, nullptr,
                                         gens, s);
        return ee;
    };
    // two warm-up generations, then the state every candidate starts from
    e = launch(cand[0], 2);
    if (e == hipSuccess) e = launch_finish(d_desc, 1, nullptr, 2, nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(backup, arena, L.total, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "tuning warm-up");
        cleanup();
        return rc;
    }
    auto time_one = [&](Entry& c) -> int {
        hipError_t ee = hipMemcpyAsync(arena, backup, L.total, hipMemcpyDeviceToDevice, s);
        if (ee == hipSuccess) ee = hipEventRecord(e0, s);
        if (ee == hipSuccess) ee = launch(c, trial_generations);
        if (ee == hipSuccess) ee = hipEventRecord(e1, s);
        if (ee == hipSuccess) ee = hipEventSynchronize(e1);
        float f = 0.f;
        if (ee == hipSuccess) ee = hipEventElapsedTime(&f, e0, e1);
        if (ee != hipSuccess) return hip_fail(ee, "tuning launch");
        c.ms = std::min(c.ms, (double)f / trial_generations);
        return QIEO_OK;
    };
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t j = 0; j < cand.size(); ++j) {
            Entry& c = cand[pass == 0 ? j : cand.size() - 1 - j];
            if ((rc = time_one(c))) {
                cleanup();
                return rc;
            }
        }
    }
    cleanup();
    Entry best{0, 0, 0, 1e300};
    double worst = 0.0;
    for (auto& c : cand) {
        if (c.ms < best.ms) best = c;
        worst = std::max(worst, c.ms);
    }
    {
        std::lock_guard<std::mutex> lk(g_db_mu);
        g_db[instance_key(n_pop, L.nchunk)] = best;
    }
    if (out) {
        out->rows_per_block = best.R;
        out->waves_per_block = best.S;
        out->flags = best.flags;
        out->ms_per_generation = best.ms;
        out->worst_ms_per_generation = worst;
        out->candidates = (int32_t)cand.size();
    }
    return QIEO_OK;
}

extern "C" int qieo_tune_db_save(const char* path)
{
    clear_error();
    if (!path) return set_error(QIEO_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(QIEO_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_db_mu);
    std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [");
    bool first = true;
    for (auto& kv : g_db) {
        int kind, a, b, c;
        std::tie(kind, a, b, c) = kv.first;
        if (kind == 0)
            std::fprintf(f, "%s\n  {\"np_log2\": %d, \"nchunk_log2\": %d, \"R\": %d, \"S\": %d, "
                            "\"flags\": %d, \"ms\": %.6f}",
                         first ? "" : ",", a, b, kv.second.R, kv.second.S, kv.second.flags,
                         kv.second.ms);
        else
            std::fprintf(f, "%s\n  {\"class\": %d, \"rows_log2\": %d, \"nchunk_log2\": %d, "
                            "\"R\": %d, \"S\": %d, \"flags\": %d, \"ms\": %.6f}",
                         first ? "" : ",", a, b, c, kv.second.R, kv.second.S, kv.second.flags,
                         kv.second.ms);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    std::fclose(f);
    return QIEO_OK;
}

// Reads the file written by qieo_tune_db_save (one entry object per line).
extern "C" int qieo_tune_db_load(const char* path)
{
    clear_error();
    if (!path) return set_error(QIEO_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_error(QIEO_EINVAL, "cannot read %s", path);
    char line[512];
    int n = 0;
    std::map<Key, Entry> loaded;
    while (std::fgets(line, sizeof line, f)) {
        int a, b, c = 0, R, S, fl;
        double ms;
        Key key;
        const char* p;
        if ((p = std::strstr(line, "\"np_log2\""))) {
            if (std::sscanf(p, "\"np_log2\": %d, \"nchunk_log2\": %d, \"R\": %d, \"S\": %d, "
                               "\"flags\": %d, \"ms\": %lf", &a, &b, &R, &S, &fl, &ms) != 6)
                continue;
            key = Key{0, a, b, 0};
        } else if ((p = std::strstr(line, "\"class\""))) {
            if (std::sscanf(p, "\"class\": %d, \"rows_log2\": %d, \"nchunk_log2\": %d, \"R\": %d, "
                               "\"S\": %d, \"flags\": %d, \"ms\": %lf",
                            &a, &b, &c, &R, &S, &fl, &ms) != 7)
                continue;
            if (a < -1 || a >= kClasses) continue;
            key = Key{1, a, b, c};
            // class -1: a batch's on-chip variant subset (R = its launches,
            // S = waves per workgroup, flags = the subset)
            if (a == -1) {
                if (R < 1 || S != kOnchipWaves || fl < 1 || fl >= (1 << kOnchipVariants)) continue;
                loaded[key] = Entry{R, S, fl, ms};
                ++n;
                continue;
            }
        } else {
            continue;
        }
        if ((R != 1 && R != 2 && R != 4) || S < 1 || S > 16 || fl < 0 || fl > kFlagAll) continue;
        loaded[key] = Entry{R, S, fl, ms};
        ++n;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_db_mu);
    for (auto& kv : loaded) g_db[kv.first] = kv.second;
    return n;
}

extern "C" void qieo_tune_db_clear(void)
{
    std::lock_guard<std::mutex> lk(g_db_mu);
    g_db.clear();
}
