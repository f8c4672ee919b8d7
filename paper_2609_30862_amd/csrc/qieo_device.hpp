// Device building blocks of the QIEO generation for gfx950 (CDNA4, wave64).
//
// Everything here is per-lane arithmetic; the layout and control flow live in
// qieo_kernels.hip.  Floating-point expressions are written one IEEE binary32
// operation at a time and the library is compiled with -ffp-contract=off, so
// no multiply is fused into an add.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qieo_layout.hpp"

namespace qieo {

// ---------------------------------------------------------------------------
// Rotation-gate constants: binary32 roundings of cos(0.01 pi), sin(0.01 pi)
// and the initial amplitude 1/sqrt(2).
// ---------------------------------------------------------------------------
constexpr float kCos = 0x1.ffbf52p-1f;
constexpr float kSin = 0x1.015122p-5f;
constexpr float kAmp0 = 0x1.6a09e6p-1f;

// The same three constants for binary64 amplitudes: correctly rounded
// binary64 values of cos(0.01 pi), sin(0.01 pi) and 1/sqrt(2).
template <typename T> struct Gate;
template <> struct Gate<float> {
    static constexpr float c = 0x1.ffbf52p-1f, s = 0x1.015122p-5f, a0 = 0x1.6a09e6p-1f;
};
template <> struct Gate<double> {
    static constexpr double c = 0x1.ffbf52e9d1086p-1, s = 0x1.015122df75860p-5,
                            a0 = 0x1.6a09e667f3bcdp-1;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  The key is wave-uniform (it is the
// instance seed) and so is every round's key; counter word 0 is the only
// per-lane input, words 1-3 (chromosome, generation, stream 0) are uniform.
// The 32x32->64 products are plain 64-bit multiplies, which the compiler
// lowers to v_mad_u64_u32 for per-lane operands and to scalar multiplies for
// uniform ones.
// ---------------------------------------------------------------------------
struct Draw4 {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ void philox_round(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                             uint32_t& x3, uint32_t k0, uint32_t k1)
{
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    const uint32_t y1 = (uint32_t)pb;
    const uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    const uint32_t y3 = (uint32_t)pa;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
}

// a ^ b ^ k in one instruction (gfx950's three-input bitwise operation,
// truth table 0x96), for per-lane a, b and a wave-uniform k
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t k, uint32_t b)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "s"(k), "v"(b));
    return r;
}

// A round whose four words are all per-lane: the same arithmetic as
// philox_round, each word's two XORs in one instruction.
__device__ __forceinline__ void philox_round_lanes(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                                   uint32_t& x3, uint32_t k0, uint32_t k1)
{
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = xor3((uint32_t)(pb >> 32), k0, x1);
    const uint32_t y1 = (uint32_t)pb;
    const uint32_t y2 = xor3((uint32_t)(pa >> 32), k1, x3);
    const uint32_t y3 = (uint32_t)pa;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
}

__device__ __forceinline__ Draw4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
    // The round keys are two scalar adds each; left loop-invariant, the
    // compiler would keep all twenty in scalar registers across a kernel's
    // chunk loop (and spill them once registers are tight), so the key is
    // passed through an empty asm here, which makes each call derive its own.
    asm volatile("" : "+s"(k0), "+s"(k1));
    // The first two Philox rounds still have uniform words (only counter
    // word 0 is per-lane at the start), which the compiler keeps scalar;
    // from the third on every word is per-lane.
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r < 2) philox_round(c0, c1, c2, c3, k0, k1);
        else philox_round_lanes(c0, c1, c2, c3, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Draw4{c0, c1, c2, c3};
}

// Keeps a chunk's draws where they are computed: an empty asm that uses
// them, so the compiler issues the Philox arithmetic before the code that
// follows (the rotation, which first waits for the allele masks' scalar
// loads) instead of sinking it down to the observation that reads it.
__device__ __forceinline__ void pin_draws(const Draw4& d)
{
    asm volatile("" ::"v"(d.r0), "v"(d.r1), "v"(d.r2), "v"(d.r3));
}

// Observation of one qubit: 1 iff the 24-bit uniform of r lies below beta^2
// (the uniform is exact in either precision).
template <typename T>
__device__ __forceinline__ bool observe(uint32_t r, T beta)
{
    const T u = (T)(r >> 8) * (T)0x1p-24;
    const T b2 = beta * beta;
    return u < b2;
}

// ---------------------------------------------------------------------------
// Lane-mask helpers.  A wave-uniform 64-bit mask m holds one bit per lane;
// sel(m, f, t) returns t on lanes whose bit is set and f elsewhere, in a
// single v_cndmask_b32 with m as the SGPR-pair condition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t uniform_mask(uint64_t m)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)m);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(m >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ float sel(uint64_t m, float if0, float if1)
{
    float r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(if0), "v"(if1), "s"(uniform_mask(m)));
    return r;
}

__device__ __forceinline__ uint32_t sel(uint64_t m, uint32_t if0, uint32_t if1)
{
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(if0), "v"(if1), "s"(uniform_mask(m)));
    return r;
}

__device__ __forceinline__ double sel(uint64_t m, double if0, double if1)
{
    const uint64_t a = __builtin_bit_cast(uint64_t, if0), b = __builtin_bit_cast(uint64_t, if1);
    uint32_t lo, hi;
    const uint64_t mm = uniform_mask(m);
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(lo) : "v"((uint32_t)a), "v"((uint32_t)b), "s"(mm));
    asm("v_cndmask_b32 %0, %1, %2, %3"
        : "=v"(hi) : "v"((uint32_t)(a >> 32)), "v"((uint32_t)(b >> 32)), "s"(mm));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Memory helpers.  Streams of the amplitude planes use global (address space
// 1) vector loads/stores from a wave-uniform row base plus a 32-bit per-lane
// index; wave-uniform reads of allele words use the constant address space
// so they become scalar loads into SGPRs.  The kernels never write memory they
// read through the scalar path within the same launch.
// ---------------------------------------------------------------------------
#define QIEO_AS_GLOBAL __attribute__((address_space(1)))
#define QIEO_AS_CONST __attribute__((address_space(4)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef f32x4 type; };
template <> struct Vec4<double> { typedef f64x4 type; };

template <typename T>
__device__ __forceinline__ T gload(const T* base, uint32_t idx)
{
    return ((const QIEO_AS_GLOBAL T*)base)[idx];
}

template <typename T>
__device__ __forceinline__ void gstore(T* base, uint32_t idx, T v)
{
    ((QIEO_AS_GLOBAL T*)base)[idx] = v;
}

// Streaming load of data this launch reads once (no L2 retention).
template <typename T>
__device__ __forceinline__ T gload_nt(const T* base, uint32_t idx)
{
    return __builtin_nontemporal_load(&((const QIEO_AS_GLOBAL T*)base)[idx]);
}

// Streaming store that is not expected to be re-read soon (no L2 retention).
template <typename T>
__device__ __forceinline__ void gstore_nt(T* base, uint32_t idx, T v)
{
    __builtin_nontemporal_store(v, &((QIEO_AS_GLOBAL T*)base)[idx]);
}

template <typename T>
__device__ __forceinline__ T sload(const T* p)
{
    return *(const QIEO_AS_CONST T*)p;
}

// ---------------------------------------------------------------------------
// Wave64 reductions through DPP lane moves (quad permutes, row mirrors, then
// the row broadcasts of lane 15 and 31), which stay in registers; the
// complete result ends in lane 63 and is read from there.  Integer sums and
// maxima do not depend on the order of combination.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    // lanes outside ROWS, or whose source is out of range, receive 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_sum_dpp(uint32_t v)
{
    v += dpp_u32<0xb1, 0xf>(v);       // quad_perm [1,0,3,2]: pairs
    v += dpp_u32<0x4e, 0xf>(v);       // quad_perm [2,3,0,1]: quads
    v += dpp_u32<0x141, 0xf>(v);      // row_half_mirror: 8 lanes
    v += dpp_u32<0x140, 0xf>(v);      // row_mirror: 16-lane rows
    v += dpp_u32<0x142, 0xa>(v);      // row_bcast:15 into rows 1, 3
    v += dpp_u32<0x143, 0xc>(v);      // row_bcast:31 into rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_u64(uint64_t v)
{
    const uint64_t lo = dpp_u32<CTRL, ROWS>((uint32_t)v);
    const uint64_t hi = dpp_u32<CTRL, ROWS>((uint32_t)(v >> 32));
    const uint64_t o = (hi << 32) | lo;
    return o > v ? o : v;
}

__device__ __forceinline__ uint64_t wave_max_u64_dpp(uint64_t v)
{
    v = dpp_max_u64<0xb1, 0xf>(v);
    v = dpp_max_u64<0x4e, 0xf>(v);
    v = dpp_max_u64<0x141, 0xf>(v);
    v = dpp_max_u64<0x140, 0xf>(v);
    v = dpp_max_u64<0x142, 0xa>(v);
    v = dpp_max_u64<0x143, 0xc>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t ballot(bool p)
{
    return __ballot(p);
}

// Loads a 64-bit lane mask that every lane reads from the same address and
// pins it to scalar registers.
__device__ __forceinline__ uint64_t load_mask(const uint64_t* p)
{
    return sload(p);
}

// ---------------------------------------------------------------------------
// CIP on one gene, given as lane masks: rot = lanes whose gene must move
// toward the elite, tgt = lanes whose elite allele is 1.  Direction: positive
// angle raises beta^2 when alpha*beta > 0, so the step is +0.01 pi toward 1
// and -0.01 pi toward 0 when the product is positive, the opposite when it is
// negative; a zero product steps by +0.01 pi unless the gene already sits on
// the target pole (target 1 with alpha == 0, target 0 with beta == 0).  The
// sign logic runs on the comparisons' lane masks in scalar registers; the
// pole test is needed only when a moving lane has a zero product, which the
// wave decides once.  The Newton factor g = 1.5 - 0.5 n pulls the norm back
// to 1: 0.5 n is exact (a halving; a subnormal n leaves 1.5 - 0.5 n = 1.5
// either way), so the fused g = fma(-0.5, n, 1.5) rounds once to the same
// value as the two separately rounded operations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ void cip_gene(T& a, T& b, uint64_t rot, uint64_t tgt)
{
    constexpr T kC = Gate<T>::c, kS = Gate<T>::s;
    const T p = a * b;
    const uint64_t pos = ballot(p > (T)0), neg = ballot(p < (T)0);
    const uint64_t minus = (pos & ~tgt) | (neg & tgt);
    const T sd = sel(minus, kS, -kS);
    uint64_t mv = rot;
    if ((rot & ~(pos | neg)) != 0) {
        const T pole = sel(tgt, b, a);
        mv &= ~ballot(pole == (T)0);
    }
    const T ca = kC * a;
    const T sb = sd * b;
    const T a1 = ca - sb;
    const T sa = sd * a;
    const T cb = kC * b;
    const T b1 = sa + cb;
    const T aa = a1 * a1;
    const T bb = b1 * b1;
    const T n = aa + bb;
    const T g = fma_((T)-0.5, n, (T)1.5);
    const T a2 = a1 * g;
    const T b2 = b1 * g;
    a = sel(mv, a, a2);
    b = sel(mv, b, b2);
}

// CIP on a lane's four genes (slot j of the chunk in component j): the same
// gate as cip_gene, arranged so that one chunk is one straight run of code.
// The sign logic of all four genes comes first; the pole test (a moving lane
// with a zero product) is one branch for the whole chunk, almost never
// taken; then the four rotations.  A wave whose masks are all zero (a row
// that does not rotate) computes the rotations and keeps the old values.
template <typename V4, typename T>
__device__ __forceinline__ void cip_chunk(V4& a4, V4& b4, const uint64_t rot[4],
                                          const uint64_t tgt[4])
{
    constexpr T kC = Gate<T>::c, kS = Gate<T>::s;
    T a[4] = {a4.x, a4.y, a4.z, a4.w};
    T b[4] = {b4.x, b4.y, b4.z, b4.w};
    T sd[4];
    uint64_t mv[4];
    uint64_t zero = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const T p = a[j] * b[j];
        const uint64_t pos = ballot(p > (T)0), neg = ballot(p < (T)0);
        sd[j] = sel((pos & ~tgt[j]) | (neg & tgt[j]), kS, -kS);
        mv[j] = rot[j];
        zero |= rot[j] & ~(pos | neg);
    }
    if (zero != 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) mv[j] &= ~ballot(sel(tgt[j], b[j], a[j]) == (T)0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const T ca = kC * a[j];
        const T sb = sd[j] * b[j];
        const T a1 = ca - sb;
        const T sa = sd[j] * a[j];
        const T cb = kC * b[j];
        const T b1 = sa + cb;
        const T aa = a1 * a1;
        const T bb = b1 * b1;
        const T n = aa + bb;
        const T g = fma_((T)-0.5, n, (T)1.5);
        a[j] = sel(mv[j], a[j], a1 * g);
        b[j] = sel(mv[j], b[j], b1 * g);
    }
    a4 = V4{a[0], a[1], a[2], a[3]};
    b4 = V4{b[0], b[1], b[2], b[3]};
}

// The alleles of one 256-gene chunk, four 64-bit wave masks (slot j of every
// lane), stored as eight words: lane l < 8 holds word l (half l & 1 of mask
// l >> 1), written into its lane from the scalar registers, so the chunk's
// 32 bytes go out in one store instruction.  Lanes 8..63 of the result are
// not used.
template <int L>
__device__ __forceinline__ void write_lane(uint32_t& w, uint32_t v)
{
    asm("v_writelane_b32 %0, %1, %2" : "+v"(w) : "s"(v), "n"(L));
}

__device__ __forceinline__ uint32_t chunk_word(uint64_t m0, uint64_t m1, uint64_t m2,
                                               uint64_t m3)
{
    uint32_t w = 0u;
    write_lane<0>(w, (uint32_t)uniform_mask(m0));
    write_lane<1>(w, (uint32_t)(uniform_mask(m0) >> 32));
    write_lane<2>(w, (uint32_t)uniform_mask(m1));
    write_lane<3>(w, (uint32_t)(uniform_mask(m1) >> 32));
    write_lane<4>(w, (uint32_t)uniform_mask(m2));
    write_lane<5>(w, (uint32_t)(uniform_mask(m2) >> 32));
    write_lane<6>(w, (uint32_t)uniform_mask(m3));
    write_lane<7>(w, (uint32_t)(uniform_mask(m3) >> 32));
    return w;
}

__device__ __forceinline__ void store_chunk_words(uint32_t* dst, uint64_t m0, uint64_t m1,
                                                  uint64_t m2, uint64_t m3, int lane)
{
    const uint32_t word = chunk_word(m0, m1, m2, m3);
    if (lane < kWordsPerChunk) gstore(dst, (uint32_t)lane, word);
}

// Evaluation's per-lane sum of eq. (1) over the lane's four genes: the items
// of the genes whose allele bit is set in the masks.
__device__ __forceinline__ uint32_t masked_sum4(uint64_t m0, uint64_t m1, uint64_t m2,
                                                uint64_t m3, i32x4 v)
{
    return sel(m0, 0u, (uint32_t)v.x) + sel(m1, 0u, (uint32_t)v.y) + sel(m2, 0u, (uint32_t)v.z) +
           sel(m3, 0u, (uint32_t)v.w);
}

// The same gate for one gene owned by one lane (chromosome-parallel mapping):
// identical operations in identical order, selected per lane instead of by
// wave masks, so both mappings produce the same bits.
__device__ __forceinline__ void cip_gene_lane(float& a, float& b, bool tgt)
{
    const float p = a * b;
    float sd = tgt ? kSin : -kSin;
    if (p < 0.0f) sd = tgt ? -kSin : kSin;
    else if (!(p > 0.0f)) sd = kSin;
    const bool skip = (tgt ? a : b) == 0.0f;
    const float ca = kCos * a;
    const float sb = sd * b;
    const float a1 = ca - sb;
    const float sa = sd * a;
    const float cb = kCos * b;
    const float b1 = sa + cb;
    const float aa = a1 * a1;
    const float bb = b1 * b1;
    const float n = aa + bb;
    const float hn = 0.5f * n;
    const float g = 1.5f - hn;
    if (!skip) {
        a = a1 * g;
        b = b1 * g;
    }
}

}  // namespace qieo
