// Host-side helpers shared by the single-instance, batch and server runtimes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/qieo.h"
#include "qieo_host.hpp"
#include "qieo_kernels.hpp"

namespace qieo {

int hip_fail(hipError_t e, const char* what);

// Device memory through the caller's allocator when a qieo_dev_ctx gives
// one, else hipMalloc / hipFree.
struct DevMem {
    qieo_dev_ctx ctx{};
    bool custom = false;
    void set(const qieo_dev_ctx* c)
    {
        if (c && c->alloc) {
            ctx = *c;
            custom = true;
        }
    }
    void* alloc(size_t bytes) const;    // nullptr on failure (HIP error state cleared)
    void release(void* p) const;        // nullptr is ignored
};

InstDev bind_arena(char* base, const ArenaLayout& L, int32_t ng, int32_t np, int32_t cap,
                   uint64_t seed);
int upload_and_init(const InstDev& d, const qieo_item* items, hipStream_t s,
                    const ArenaLayout& L, char* base, std::vector<int32_t>& staging,
                    bool f64 = false);
int check_device();
// hipMemcpyAsync on s, then waits for s.
hipError_t copy_on(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s);
// Shape from the autotuner's database, if the bucket was tuned.
bool tuned_tile(int32_t np, int32_t nchunk, int* R, int* S, int* flags);
// Shape of a batch's launch class (class, rows of the class, longest row in
// chunks) from the autotuner's database, if that bucket was tuned.
bool tuned_class(int cls, int64_t rows, int32_t max_nchunk, int* R, int* S, int* flags);
// Records the tuned shape of a batch's launch class in that database.
void record_class(int cls, int64_t rows, int32_t max_nchunk, int R, int S, int flags, double ms);
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
