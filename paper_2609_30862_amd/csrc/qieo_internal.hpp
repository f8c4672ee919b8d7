// Host-side helpers shared by the single-instance, batch and server runtimes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/qieo.h"
#include "qieo_kernels.hpp"

namespace qieo {

// Byte offsets of every plane inside one instance's device arena.
struct ArenaLayout {
    int32_t pitch, nchunk;
    size_t alpha, beta, xbits, v, w, fit, prof, wt, ekey, best, best_bits, tbase, conv, part;
    size_t zero_from;
    size_t total;
};

int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
void clear_error();

// elem: bytes per amplitude (4 binary32, 8 binary64)
size_t arena_layout(int32_t ng, int32_t np, ArenaLayout* L, int elem = 4);
InstDev bind_arena(char* base, const ArenaLayout& L, int32_t ng, int32_t np, int32_t cap,
                   uint64_t seed);
// n_items in [1, 2^30 - 256], n_pop >= 1, at most 2^36 genes (rows padded to 64)
int validate_shape(int32_t n_items, int32_t n_pop);
int validate_problem(const qieo_item* items, int32_t n_items, int32_t capacity, int32_t n_pop);
int upload_and_init(const InstDev& d, const qieo_item* items, hipStream_t s,
                    const ArenaLayout& L, char* base, std::vector<int32_t>& staging,
                    bool f64 = false);
int check_device();
void pick_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags, int elem_bytes = 4);
// hipMemcpyAsync on s, then waits for s.
hipError_t copy_on(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s);
// kFlag* bits for a work shape given the amplitude bytes one generation streams.
int variant_flags(int R, int S, int64_t nchunk, int64_t plane_bytes);
// Shape from the autotuner's database, if the bucket was tuned.
bool tuned_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags);
int read_best(const InstDev& d, int32_t capacity, hipStream_t s, qieo_result* out,
              uint32_t* bits, size_t n_words);
int export_rows(const InstDev& d, const InstDev* d_desc, hipStream_t s,
                int32_t row0, int32_t n_rows, void* alpha, void* beta, uint8_t* alleles,
                int32_t* fitness, int32_t* profit, int32_t* weight, int32_t* elite,
                bool f64 = false);
int read_generations(const InstDev& d, hipStream_t s, int64_t* t);
int read_convergence(const InstDev& d, hipStream_t s, int32_t* converged, int64_t* generation);
int write_window(const InstDev& d, hipStream_t s, int32_t window);

}  // namespace qieo
