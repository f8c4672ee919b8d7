// DetermineElite's device side (Sec. III-B): the 64-bit elite key, the offer
// of a row's key to its generation's slot, and the best-so-far record.
// Shared by every kernel that closes a generation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qieo_layout.hpp"

namespace qieo {

// key = ((uint32)f ^ 0x80000000) << 32 | ~row: the largest key is the
// largest fitness, lowest row among equals (the paper's lowest-index tie
// rule for the argmax).
__device__ __forceinline__ int32_t key_fitness(unsigned long long key)
{
    return (int32_t)((uint32_t)(key >> 32) ^ 0x80000000u);
}

__device__ __forceinline__ int32_t key_row(unsigned long long key)
{
    return (int32_t)(~(uint32_t)key);
}

__device__ __forceinline__ unsigned long long make_key(int32_t f, int32_t row)
{
    return ((unsigned long long)((uint32_t)f ^ 0x80000000u) << 32) |
           (unsigned long long)(~(uint32_t)row);
}

// Offers a row's key to the generation's elite slot.  Device-scope atomics
// on one address serialise at the memory side (about 12 ns per wave
// instruction on MI355X: 4096 rows cost 48 us), so the slot is read first
// and the atomic issued only by a key that can still win; the slot only
// grows during a generation, so a key not above a value once read is never
// the maximum and skipping it leaves the result unchanged.
__device__ __forceinline__ void offer_key(unsigned long long* slot, unsigned long long key)
{
    const unsigned long long cur = __hip_atomic_load(slot, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    if (key > cur) atomicMax(slot, key);
}

// Best-so-far update for generation tg whose elite is (e, fe).  Executed by
// one whole wavefront (the only writer of the record at that point), once
// generation tg is complete.
__device__ inline void best_update(const InstDev& I, int64_t tg, int32_t e, int32_t fe,
                                   const uint32_t* __restrict__ xg, int lane)
{
    const int has = I.best[0];
    const int32_t bf = I.best[1];
    if (has && !(fe > bf)) return;
    const int wpr = I.nchunk * kWordsPerChunk;
    const uint32_t* src = xg + (size_t)e * wpr;
    for (int i = lane; i < wpr; i += 64) I.best_bits[i] = src[i];
    if (lane == 0) {
        const int slot = (int)(tg & 1) * I.np + e;
        I.best[1] = fe;
        I.best[2] = I.prof[slot];
        I.best[3] = I.wt[slot];
        I.best[4] = (int32_t)(uint32_t)(uint64_t)tg;
        I.best[5] = (int32_t)(uint32_t)((uint64_t)tg >> 32);
        I.best[6] = e;
        I.best[0] = 1;
    }
}

}  // namespace qieo
