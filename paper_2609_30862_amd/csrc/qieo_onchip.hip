// On-chip loop: one cooperative launch runs every generation of a call for a
// population whose amplitude planes fit in the chip's registers.
//
// Per-generation launches stream alpha and beta through the caches every
// generation (16 bytes a gene in binary32).  Here they stay in registers for
// the whole call: one workgroup of 16 waves per CU (all resident at once,
// which the cooperative launch guarantees), workgroup b owning rows
// [b*R, b*R + R) whole, wave w holding the workgroup's (row, chunk) items
// w*K .. w*K + K - 1 in row-major order, four genes of each per lane, i.e.
// 8K registers of amplitudes.  A generation is the fused one of the
// per-generation kernels, gene for gene the same arithmetic (so the same
// bits): CIP(t-1) toward the elite of t-1, QIP(t), Evaluation's sums of
// eq. (1) closed per row inside the workgroup, and the row's key offered to
// the elite slot of t.  A grid barrier then ends the generation; after it
// the elite of t is final everywhere.
//
// Item tables, the workgroup's own allele words of t-1 and t, and the elite's
// words of t-1 are read from LDS.  Allele words, fitness slots, elite keys
// and the best-so-far record go to global memory exactly as the
// per-generation launches write them (the elite's words and the best record
// are read back from there by other workgroups); the planes are written
// once, at the end.  The call therefore leaves the state the per-generation
// launches would leave, and the next call (of any kind) continues from it.
//
// Grid barrier: an arrival counter in the instance's arena (cleared by a
// small launch before this one).  Each workgroup waits for its own stores,
// then one thread adds its arrival with release semantics at device scope
// (the XCD's L2 writes back what the workgroup wrote) and spins on the
// counter; once it reaches the generation's target, an acquire at device
// scope drops stale lines before anyone reads other workgroups' data.  The
// wait is bounded in time: past the bound the waiting workgroup raises the
// abort flag, every workgroup that sees it leaves, and the host reports the
// call as failed (the state is then undefined).
#include <mutex>

#include "qieo_device.hpp"
#include "qieo_elite.hpp"
#include "qieo_host.hpp"
#include "qieo_kernels.hpp"

namespace qieo {

namespace {

// Four 64-bit lane masks from the eight allele words at p (LDS), as
// wave-uniform values: lane j reads word j, then the words are read out of
// lanes 0..7.
__device__ __forceinline__ void lds_masks(const uint32_t* p, int lane, uint64_t m[4])
{
    const uint32_t w = p[lane & (kWordsPerChunk - 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)w, 2 * j);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)w, 2 * j + 1);
        m[j] = ((uint64_t)hi << 32) | lo;
    }
}

// Ends a generation for the whole grid.  Returns false if the wait ran past
// its bound or another workgroup gave up (every thread gets the same answer).
__device__ __forceinline__ bool grid_barrier(uint32_t* sync, uint32_t target, int64_t spin_ticks,
                                             int* s_flag)
{
    // this wave's stores (allele words, fitness, best record) have reached
    // the L2 before the workgroup's arrival can be counted
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int bad = 0;
        const int64_t start = wall_clock64();
        while ((int32_t)(__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                         target) < 0) {
            if (__hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                bad = 1;
                break;
            }
            if (wall_clock64() - start > spin_ticks) {
                __hip_atomic_store(sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bad = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = bad;
    }
    __syncthreads();
    return *s_flag == 0;
}

__global__ void onchip_reset_kernel(const InstDev* __restrict__ insts)
{
    if (threadIdx.x < 2) insts[0].sync[threadIdx.x] = 0u;
}

template <int K>
__global__ __launch_bounds__(64 * kOnchipWaves) void onchip_kernel(const InstDev* __restrict__ insts,
                                                                  int R, int gens,
                                                                  int64_t spin_ticks)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int s_flag;
    const InstDev I = insts[0];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int np = I.np, pitch = I.pitch, nchunk = I.nchunk, wpr = nchunk * kWordsPerChunk;
    const int row0 = (int)blockIdx.x * R;
    const int nrows = min(R, np - row0);            // >= 1: the grid is ceil(np / R)
    const int n_items = nrows * nchunk;

    int32_t* sV = reinterpret_cast<int32_t*>(lds);                     // [nchunk * 256]
    int32_t* sWt = sV + nchunk * kChunk;                                 // [nchunk * 256]
    uint32_t* sX = reinterpret_cast<uint32_t*>(sWt + nchunk * kChunk);   // [2][R][wpr] by parity
    uint32_t* sE = sX + 2 * R * wpr;                                     // [wpr] elite of t-1
    int32_t* sF = reinterpret_cast<int32_t*>(sE + wpr);                  // [2][R] fitness by parity
    uint32_t* sSum = reinterpret_cast<uint32_t*>(sF + 2 * R);            // [R][2] profit, weight

    const int64_t t0 = sload(I.tbase);
    // item tables, and the rows' allele words and fitness of t0 - 1 (for
    // t0 = 0 the zeroed slot 1, which nothing uses: no row rotates at 0)
    for (int i = tid; i < nchunk * kChunk; i += nthr) {
        sV[i] = I.v[i];
        sWt[i] = I.w[i];
    }
    {
        const int pp = (int)((t0 - 1) & 1);
        const uint32_t* src = I.xbits + ((size_t)pp * np + row0) * wpr;
        for (int i = tid; i < nrows * wpr; i += nthr) sX[pp * R * wpr + i] = src[i];
        if (tid < nrows) sF[pp * R + tid] = I.fit[pp * np + row0 + tid];
        if (tid < 2 * R) sSum[tid] = 0u;
    }

    // the wave's first item and its amplitudes; lanes past a row's end
    // (part of its last chunk) read the next row or the plane's slack and
    // are never observed, rotated or stored
    const int first = wave * K;
    const int r_first = first / nchunk, ch_first = first - r_first * nchunk;
    // Every wave runs K items; a wave with fewer real ones (the last waves
    // of a workgroup whose rows do not fill all waves) runs the rest on row
    // 0's chunks and stores nothing from them.  The amplitude registers are
    // then updated on every path, so the compiler keeps one copy of them.
    f32x4 A[K], B[K];
    {
        int r = r_first, ch = ch_first;
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const bool valid = first + u < n_items;
            const size_t base = (size_t)(row0 + (valid ? r : 0)) * pitch;
            const uint32_t q = (uint32_t)(ch * kChunk / 4) + lane;
            A[u] = gload((const f32x4*)(I.alpha + base), q);
            B[u] = gload((const f32x4*)(I.beta + base), q);
            if (++ch == nchunk) { ch = 0; ++r; }
        }
    }
    __syncthreads();

    for (int k = 0; k < gens; ++k) {
        const int64_t t = t0 + k;
        const int par = (int)(t & 1);
        const bool pending = t > 0;
        int32_t e_prev = 0, fe_prev = 0;
        if (pending) {
            // final: written by the previous launch, or before the last barrier
            const unsigned long long key = __hip_atomic_load(I.ekey + (t - 1) % 3, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
            e_prev = __builtin_amdgcn_readfirstlane(key_row(key));
            fe_prev = __builtin_amdgcn_readfirstlane(key_fitness(key));
        }
        const uint32_t* xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
        uint32_t* xcur = I.xbits + (size_t)par * np * wpr;
        // the previous generation's bookkeeping, as the first workgroup of a
        // per-generation launch does it (no convergence window here)
        if (blockIdx.x == 0 && wave == 0) {
            if (pending) best_update(I, t - 1, e_prev, fe_prev, xprev, lane);
            if (lane == 0)
                __hip_atomic_store(I.ekey + (t + 1) % 3, 0ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (pending)
            for (int i = tid; i < wpr; i += nthr) sE[i] = xprev[(size_t)e_prev * wpr + i];
        __syncthreads();

        const uint32_t* sXp = sX + (par ^ 1) * R * wpr;
        uint32_t* sXc = sX + par * R * wpr;
        uint32_t accP = 0u, accW = 0u;
        // the item coordinates pass through an empty asm, so nothing derived
        // from them is computed once and held across the generation loop
        int r = r_first, ch = ch_first, fi = first, ni = n_items;
        asm volatile("" : "+s"(r), "+s"(ch), "+s"(fi), "+s"(ni));
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const bool valid = fi + u < ni;
            // One item at a time: the scheduler would otherwise hoist later
            // items' loads and draws, and the per-item values that do not
            // change between generations (addresses, the lane's counter
            // word, the first Philox round's products) would be kept for
            // every item across the generation loop.  The lane index passes
            // through an empty asm, so they are derived again here.
            __builtin_amdgcn_sched_barrier(0);
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int rv = valid ? r : 0;
            const int c = row0 + rv;
            const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * (uint32_t)ln;
            const uint64_t actm = ballot(g0 < (uint32_t)pitch);
            const uint32_t q = g0 >> 2;
            // the elite's and the row's own alleles of t-1
            uint64_t bm[4], xm[4];
            lds_masks(sE + ch * kWordsPerChunk, ln, bm);
            lds_masks(sXp + rv * wpr + ch * kWordsPerChunk, ln, xm);
            const int32_t f_prev = __builtin_amdgcn_readfirstlane(sF[(par ^ 1) * R + rv]);
            const Draw4 d = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
            pin_draws(d);
            // genes that move: the row scores below the elite and the allele
            // differs from the elite's
            const uint64_t rowm = (pending && f_prev < fe_prev) ? ~0ull : 0ull;
            const uint64_t mv[4] = {(xm[0] ^ bm[0]) & rowm, (xm[1] ^ bm[1]) & rowm,
                                    (xm[2] ^ bm[2]) & rowm, (xm[3] ^ bm[3]) & rowm};
            cip_chunk<f32x4, float>(A[u], B[u], mv, bm);
            const uint64_t m0 = ballot(observe(d.r0, B[u].x)) & actm;
            const uint64_t m1 = ballot(observe(d.r1, B[u].y)) & actm;
            const uint64_t m2 = ballot(observe(d.r2, B[u].z)) & actm;
            const uint64_t m3 = ballot(observe(d.r3, B[u].w)) & actm;
            const uint32_t word = chunk_word(m0, m1, m2, m3);
            if (valid && lane < kWordsPerChunk) {
                gstore(xcur + (size_t)c * wpr + ch * kWordsPerChunk, (uint32_t)lane, word);
                sXc[rv * wpr + ch * kWordsPerChunk + lane] = word;
            }
            // the item tables hold nchunk * 256 entries: g0 is inside
            const i32x4 v4 = *reinterpret_cast<const i32x4*>(sV + g0);
            const i32x4 w4 = *reinterpret_cast<const i32x4*>(sWt + g0);
            accP += masked_sum4(m0, m1, m2, m3, v4);
            accW += masked_sum4(m0, m1, m2, m3, w4);
            // the row's sums go to LDS where the wave's run of it ends
            const bool row_end = ch + 1 == nchunk;
            if (valid && (row_end || u == K - 1 || fi + u + 1 == ni)) {
                const uint32_t p = wave_sum_dpp(accP), w = wave_sum_dpp(accW);
                if (lane == 0) {
                    atomicAdd(&sSum[2 * r], p);
                    atomicAdd(&sSum[2 * r + 1], w);
                }
                accP = 0u;
                accW = 0u;
            }
            if (row_end) { ch = 0; ++r; } else { ++ch; }
        }
        __syncthreads();
        // Evaluation closes per row; DetermineElite offers the row's key
        if (tid < nrows) {
            const int32_t Pi = (int32_t)sSum[2 * tid], Wi = (int32_t)sSum[2 * tid + 1];
            sSum[2 * tid] = 0u;
            sSum[2 * tid + 1] = 0u;
            const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
            sF[par * R + tid] = f;
            const int c = row0 + tid;
            const int slot = par * np + c;
            I.fit[slot] = f;
            I.prof[slot] = Pi;
            I.wt[slot] = Wi;
            offer_key(&I.ekey[t % 3], make_key(f, c));
        }
        if (k + 1 == gens) {
            // the planes as the per-generation launches leave them (rotation
            // of the last generation pending); written inside the loop, so
            // the amplitude registers are not live past it
            int rw = r_first, cw = ch_first, lw = lane;
            asm volatile("" : "+s"(rw), "+s"(cw), "+v"(lw));
#pragma unroll
            for (int u = 0; u < K; ++u) {
                const uint32_t g0 = (uint32_t)(cw * kChunk) + 4u * (uint32_t)lw;
                if (first + u < n_items && g0 < (uint32_t)pitch) {
                    const size_t base = (size_t)(row0 + rw) * pitch;
                    gstore((f32x4*)(I.alpha + base), g0 >> 2, A[u]);
                    gstore((f32x4*)(I.beta + base), g0 >> 2, B[u]);
                }
                if (++cw == nchunk) { cw = 0; ++rw; }
            }
            break;      // the launch boundary ends the last generation
        }
        if (!grid_barrier(I.sync, (uint32_t)(k + 1) * gridDim.x, spin_ticks, &s_flag)) return;
    }
}

typedef void (*OnchipFn)(const InstDev*, int, int, int64_t);

OnchipFn onchip_fn(int K)
{
    switch (K) {
        case 2: return onchip_kernel<2>;
        case 4: return onchip_kernel<4>;
        case 6: return onchip_kernel<6>;
        case 8: return onchip_kernel<8>;
        case 10: return onchip_kernel<10>;
        default: return nullptr;
    }
}

}  // namespace

// Largest dynamic LDS every variant may use on the current device, and the
// workgroups of the largest variant that fit one CU (0 if the variants
// cannot run there: no cooperative launch, or a register budget that does
// not allow one workgroup per CU).
void onchip_limits(size_t* lds_limit, int* n_cu)
{
    static std::once_flag once;
    static size_t lim = 0;
    static int cus = 0;
    std::call_once(once, [] {
        int dev = 0, coop = 0, smem = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
            hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            !coop) {
            (void)hipGetLastError();
            return;
        }
        constexpr size_t kStatic = 256;           // the kernel's own __shared__ variables
        const size_t want = (size_t)smem > kStatic ? (size_t)smem - kStatic : 0;
        for (int K : kOnchipK) {
            const void* f = reinterpret_cast<const void*>(onchip_fn(K));
            int blocks = 0;
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) !=
                    hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64 * kOnchipWaves,
                                                             want) != hipSuccess ||
                blocks < 1) {
                (void)hipGetLastError();
                return;
            }
        }
        lim = want;
        cus = ncu;
    });
    *lds_limit = lim;
    *n_cu = cus;
}

hipError_t launch_onchip(const InstDev* dI, const OnchipPlan& p, int gens, int64_t spin_ticks,
                         hipStream_t s)
{
    if (gens <= 0) return hipSuccess;
    size_t lim = 0;
    int ncu = 0;
    onchip_limits(&lim, &ncu);
    const OnchipFn f = onchip_fn(p.K);
    if (!f || p.R < 1 || p.blocks < 1 || p.blocks > ncu || p.lds > lim) return hipErrorInvalidValue;
    hipLaunchKernelGGL(onchip_reset_kernel, dim3(1), dim3(64), 0, s, dI);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const InstDev* a0 = dI;
    int a1 = p.R, a2 = gens;
    int64_t a3 = spin_ticks;
    void* args[] = {&a0, &a1, &a2, &a3};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(f), dim3((unsigned)p.blocks),
                                      dim3(64 * kOnchipWaves), args, (unsigned)p.lds, s);
}

}  // namespace qieo
