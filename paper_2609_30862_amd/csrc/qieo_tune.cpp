// Work-shape autotuner and its database.
//
// The generation kernel's speed depends on rows per workgroup R, wavefronts
// per workgroup S and the variant flags, never its results.  The tuner times
// every candidate on a scratch population of the caller's shape (its own
// arena, the caller's item tables copied device to device, the caller's
// trajectory untouched), picks the fastest, and records it under the shape's
// bucket (log2 of rows, log2 of 256-gene chunks per row).  qieo_create
// consults the database before falling back to the built-in rule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qieo.h"
#include "qieo_internal.hpp"

namespace qieo {

namespace {

struct Entry {
    int R, S, flags;
    double ms;
};

std::mutex g_db_mu;
std::map<std::pair<int, int>, Entry> g_db;

int ilog2(int64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

std::pair<int, int> bucket(int32_t np, int32_t nchunk) { return {ilog2(np), ilog2(nchunk)}; }

}  // namespace

bool tuned_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags)
{
    std::lock_guard<std::mutex> lk(g_db_mu);
    auto it = g_db.find(bucket(np, nchunk));
    if (it == g_db.end()) return false;
    *R = it->second.R;
    *S = std::min(it->second.S, std::max(1, (int)nchunk));
    *flags = it->second.flags;
    return true;
}

bool tuned_class(int cls, int64_t rows, int32_t max_nchunk, int* R, int* S, int* flags)
{
    (void)cls; (void)rows; (void)max_nchunk; (void)R; (void)S; (void)flags;
    return false;
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
        // timing does not depend on the item values: a unit-weight instance
        synth.assign((size_t)n_items, qieo_item{1, 1});
        items = synth.data();
        capacity = n_items / 2;
    }
    if ((rc = validate_problem(items, n_items, capacity, n_pop))) return rc;
    ArenaLayout L;
    arena_layout(n_items, n_pop, &L);
    char* arena = nullptr;
    InstDev* d_desc = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (arena) (void)hipFree(arena);
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
        hipMalloc((void**)&d_desc, sizeof(InstDev)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_error(QIEO_ENOMEM, "scratch population of %zu bytes does not fit", L.total);
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
            for (int f = 0; f < kFlagSegments; ++f) cand.push_back(Entry{R, S, f, 0.0});
        }
    // segment order: the work shape does not apply, only the cache hints
    for (int f : {0, kFlagNontemporal, kFlagNontemporalLoads, kFlagNontemporal | kFlagNontemporalLoads})
        cand.push_back(Entry{1, kSegWaves32, kFlagSegments | f, 0.0});
    // one generation of warm-up (generation 0 reads beta only), then trials
    auto run = [&](const Entry& c, int gens, double* ms) -> int {
        const int blocks = (n_pop + c.R - 1) / c.R;
        hipError_t ee = hipEventRecord(e0, s);
        for (int k = 0; k < gens && ee == hipSuccess; ++k)
            ee = (c.flags & kFlagSegments)
                     ? launch_segments(d_desc, n_pop, L.nchunk, L.part_nseg, c.flags, k, gens, false, s)
                     : launch_generation(d_desc, nullptr, blocks, c.R, c.S, c.flags, k, nullptr,
                                         gens, s);
        if (ee == hipSuccess) ee = launch_finish(d_desc, 1, nullptr, gens, nullptr, s);
        if (ee == hipSuccess) ee = hipEventRecord(e1, s);
        if (ee == hipSuccess) ee = hipEventSynchronize(e1);
        float f = 0.f;
        if (ee == hipSuccess) ee = hipEventElapsedTime(&f, e0, e1);
        if (ee != hipSuccess) return hip_fail(ee, "tuning launch");
        *ms = f;
        return QIEO_OK;
    };
    double tmp;
    if ((rc = run(cand[0], 1, &tmp))) {
        cleanup();
        return rc;
    }
    Entry best{0, 0, 0, 1e300};
    for (auto& c : cand) {
        if ((rc = run(c, trial_generations, &c.ms))) {
            cleanup();
            return rc;
        }
        c.ms /= trial_generations;
        if (c.ms < best.ms) best = c;
    }
    cleanup();
    {
        std::lock_guard<std::mutex> lk(g_db_mu);
        g_db[bucket(n_pop, L.nchunk)] = best;
    }
    if (out) {
        out->rows_per_block = best.R;
        out->waves_per_block = best.S;
        out->flags = best.flags;
        out->ms_per_generation = best.ms;
        double worst = 0.0;
        for (auto& c : cand) worst = std::max(worst, c.ms);
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
        std::fprintf(f, "%s\n  {\"np_log2\": %d, \"nchunk_log2\": %d, \"R\": %d, \"S\": %d, "
                        "\"flags\": %d, \"ms\": %.6f}",
                     first ? "" : ",", kv.first.first, kv.first.second, kv.second.R, kv.second.S,
                     kv.second.flags, kv.second.ms);
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
    std::map<std::pair<int, int>, Entry> loaded;
    while (std::fgets(line, sizeof line, f)) {
        int a, b, R, S, fl;
        double ms;
        const char* p = std::strstr(line, "\"np_log2\"");
        if (!p) continue;
        if (std::sscanf(p, "\"np_log2\": %d, \"nchunk_log2\": %d, \"R\": %d, \"S\": %d, "
                           "\"flags\": %d, \"ms\": %lf", &a, &b, &R, &S, &fl, &ms) != 6)
            continue;
        if ((R != 1 && R != 2 && R != 4) || S < 1 || S > 16 || fl < 0 || fl > kFlagAll) continue;
        loaded[{a, b}] = Entry{R, S, fl, ms};
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
