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
// eq. (1) closed per row inside the workgroup, and the workgroup's best key
// published.  The next generation starts in each workgroup once every
// workgroup's key is in (a grid barrier); their maximum is the elite of t.
//
// Item tables, the workgroup's own allele words of t-1 and t, and the elite's
// words of t-1 are read from LDS.  Allele words, fitness slots, elite keys
// and the best-so-far record go to global memory exactly as the
// per-generation launches write them (the elite's words and the best record
// are read back from there by other workgroups); the planes are written
// once, at the end.  The call therefore leaves the state the per-generation
// launches would leave, and the next call (of any kind) continues from it.
//
// Grid barrier and DetermineElite in one step: at the end of generation k
// each workgroup stores its best key, tagged with k, into its slot of a
// per-launch array, once its own stores have completed (the allele words,
// the only data other workgroups read during the launch, are stored at
// device scope, so completed means visible on every XCD), and at the start
// of generation k + 1 one thread per workgroup slot polls that slot until
// it carries the tag.  When
// every slot has it, the workgroup holds every workgroup's key and takes
// their maximum: the elite of k.  So no workgroup waits for a counter and
// then reads the keys, and DetermineElite needs no atomics on one address
// except in the call's last generation, whose key goes to the elite slot
// the way the per-generation launches leave it.  Data other workgroups wrote
// (the elite's allele words) is read with device-scope loads, which see the
// written-back values.  The best-so-far record is followed by every
// workgroup alike and written by the one that owns the new best row, from
// its LDS.  Waits are bounded in time: past the bound a thread raises the
// abort flag, every workgroup that sees it leaves, and the host reports the
// call as failed (the state is then undefined).
//
// Convergence window (Sec. IV-A): every workgroup knows every elite fitness
// of the call, so each counts the run of equal values that ends at the
// latest elite (seeded from the fitness ring at the start of the call) and
// all of them stop at the same generation: the one after the elite that
// completes a run of window equal values.  That generation does not run;
// the first workgroup records the stop the way the per-generation launches
// do, and the planes are written back as they stand.
#include <map>
#include <mutex>

#include "qieo_device.hpp"
#include "qieo_elite.hpp"
#include "qieo_host.hpp"
#include "qieo_kernels.hpp"
#include "qieo_onchip.hpp"

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

// A workgroup key in a slot: fitness (sign flipped), the row's complement
// in 16 bits (rows < 2^16), and the generation tag (1 .. 65535) in the low
// 16 bits.  Ordered like the elite key: larger fitness, then lower row.
__device__ __forceinline__ unsigned long long slot_key(int32_t f, int32_t row)
{
    return ((unsigned long long)((uint32_t)f ^ 0x80000000u) << 32) |
           ((unsigned long long)(~(uint32_t)row & 0xffffu) << 16);
}

__device__ __forceinline__ uint32_t slot_tag(int k) { return (uint32_t)(k % 65535) + 1u; }

// Ends generation k for the workgroup: its best key (max over wkey[], one
// per wave) goes to *slot with the tag of k, after the workgroup's stores.
__device__ __forceinline__ void publish_key(unsigned long long* slot, const unsigned long long* wkey,
                                            int nw, int k)
{
    // Every wave's stores have completed before the key is stored.  What
    // other workgroups read in this launch (the allele words, through
    // device-scope loads) was written with device-scope stores, which are
    // complete only once they are visible to every XCD; so the key needs no
    // release, whose write-back of the XCD's whole L2 (fitness slots and the
    // like, which no other workgroup reads before the launch ends) measured
    // about 1.4 us a generation.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0ull;
        for (int w = 0; w < nw; ++w) m = wkey[w] > m ? wkey[w] : m;
        __hip_atomic_store(slot, m | slot_tag(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Waits until every workgroup has published its key of generation k and
// returns their maximum (tag removed) in every thread, or false if a wait
// ran past its bound or another workgroup gave up.
__device__ __forceinline__ bool gather_keys(const unsigned long long* slots, int nb, int k,
                                            uint32_t* abort_flag, int64_t spin_ticks,
                                            unsigned long long* wkey, int* s_flag,
                                            unsigned long long* key)
{
    const int tid = threadIdx.x;
    if (tid == 0) *s_flag = 0;
    __syncthreads();
    unsigned long long m = 0ull;
    if (tid < nb) {
        const uint32_t tag = slot_tag(k);
        const int64_t start = wall_clock64();
        for (uint32_t it = 0;; ++it) {
            const unsigned long long v = __hip_atomic_load(slots + tid, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(v & 0xffffu) == tag) {
                m = v & ~0xffffull;
                break;
            }
            if ((it & 7u) == 7u &&
                __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                *s_flag = 1;
                break;
            }
            if (wall_clock64() - start > spin_ticks) {
                __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *s_flag = 1;
                break;
            }
            // no sleep between polls: each waits a memory round trip anyway,
            // and a pause only delays the sight of the key
        }
    }
    // only the polling waves hold keys: they reduce, the rest wait
    const int nwp = (nb + 63) >> 6;
    if ((tid >> 6) < nwp) {
        m = wave_max_u64_dpp(m);
        if ((tid & 63) == 0) wkey[tid >> 6] = m;
    }
    __syncthreads();
    unsigned long long r = 0ull;
    for (int w = 0; w < nwp; ++w) r = wkey[w] > r ? wkey[w] : r;
    *key = r;
    return *s_flag == 0;
}

template <typename T>
__device__ __forceinline__ T load_dev(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void store_dev(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Clears the abort flag and both generations' key slots of the launch.
__global__ void onchip_reset_kernel(const InstDev* __restrict__ insts, int nb)
{
    const InstDev I = insts[0];
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < 2) I.sync[i] = 0u;
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(I.sync + 16);
    if (i < 2 * nb) slots[i] = 0ull;
}

// The planes of the wave's K items back to global memory, from registers.
template <int K>
__device__ __forceinline__ void store_planes(const InstDev& I, const f32x4 (&A)[K],
                                             const f32x4 (&B)[K], int row0, int r, int ch,
                                             int lane, int first, int n_items)
{
    const int pitch = I.pitch, nchunk = I.nchunk;
    asm volatile("" : "+s"(r), "+s"(ch), "+v"(lane));
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * (uint32_t)lane;
        if (first + u < n_items && g0 < (uint32_t)pitch) {
            const size_t base = (size_t)(row0 + r) * pitch;
            gstore((f32x4*)(I.alpha + base), g0 >> 2, A[u]);
            gstore((f32x4*)(I.beta + base), g0 >> 2, B[u]);
        }
        if (++ch == nchunk) { ch = 0; ++r; }
    }
}

// The loop of one workgroup: rows [row0, row0 + nrows) of instance I, LDS
// laid out for R rows, workgroup blk of the nb that run the instance, gens
// generations; abort_flag is the launch's abort word.  PACKED: every profit
// and weight of the instance is at most kPackedItemMax, so the item tables
// take one LDS word per item (profit | weight << 16) and Evaluation's
// per-lane sum over four genes gives both sums at once (each half stays
// below 2^16, no carry crosses).
template <int K, bool CONV, bool PACKED>
__device__ __forceinline__ void onchip_body(const InstDev& I, const int row0, const int nrows,
                                            const int R, const int blk, const int nb,
                                            const int gens, uint32_t* abort_flag,
                                            int64_t spin_ticks)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int s_flag;
    __shared__ unsigned long long s_wkey[kOnchipWaves];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int np = I.np, pitch = I.pitch, nchunk = I.nchunk, wpr = nchunk * kWordsPerChunk;
    const int n_items = nrows * nchunk;

    int32_t* sV = reinterpret_cast<int32_t*>(lds);                     // [nchunk * 256]
    int32_t* sWt = sV + nchunk * kChunk;                                 // [nchunk * 256], not PACKED
    uint32_t* sX = reinterpret_cast<uint32_t*>(PACKED ? sWt : sWt + nchunk * kChunk);  // [2][R][wpr]
    uint32_t* sE = sX + 2 * R * wpr;                                     // [wpr] elite of t-1
    int32_t* sF = reinterpret_cast<int32_t*>(sE + wpr);                  // [2][R] fitness by parity
    int32_t* sPW = sF + 2 * R;                                           // [2][R][2] profit, weight
    uint32_t* sSum = reinterpret_cast<uint32_t*>(sPW + 4 * R);           // [R][2] running sums
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(I.sync + 16);  // [2][nb]

    const int64_t t0 = sload(I.tbase);
    // CONV: the instance has a convergence window (the launch without it
    // keeps none of the test's state in registers)
    const int window = CONV ? sload(I.conv + 3) : 0;
    if (CONV && sload(I.conv) != 0) return;         // converged in an earlier call
    // run of equal elite fitness values ending at generation t0 - 1 (counted
    // as far back as the ring reaches, which covers any window)
    int run = 0;
    int32_t run_fe = 0;
    if (CONV && t0 > 0) {
        const int lim = (int)min<int64_t>(t0, kConvRing);
        run_fe = sload(I.conv + 8 + (int)((t0 - 1) & (kConvRing - 1)));
        run = 1;
        while (run < lim && sload(I.conv + 8 + (int)((t0 - 1 - run) & (kConvRing - 1))) == run_fe)
            ++run;
    }
    // the best-so-far record as the previous launch left it; every
    // workgroup follows it the same way
    int has_best = __builtin_amdgcn_readfirstlane(I.best[0]);
    int32_t best_f = __builtin_amdgcn_readfirstlane(I.best[1]);
    // item tables, and the rows' allele words and fitness of t0 - 1 (for
    // t0 = 0 the zeroed slot 1, which nothing uses: no row rotates at 0)
    for (int i = tid; i < nchunk * kChunk; i += nthr) {
        if (PACKED) {
            sV[i] = (int32_t)((uint32_t)I.v[i] | ((uint32_t)I.w[i] << 16));
        } else {
            sV[i] = I.v[i];
            sWt[i] = I.w[i];
        }
    }
    {
        const int pp = (int)((t0 - 1) & 1);
        const uint32_t* src = I.xbits + ((size_t)pp * np + row0) * wpr;
        for (int i = tid; i < nrows * wpr; i += nthr) sX[pp * R * wpr + i] = src[i];
        if (tid < nrows) {
            sF[pp * R + tid] = I.fit[pp * np + row0 + tid];
            sPW[(pp * R + tid) * 2] = I.prof[pp * np + row0 + tid];
            sPW[(pp * R + tid) * 2 + 1] = I.wt[pp * np + row0 + tid];
        }
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

    for (int k = 0; CONV || k < gens; ++k) {
        const int64_t t = t0 + k;
        const int par = (int)(t & 1);
        const bool pending = t > 0;
        const uint32_t* sXp = sX + (par ^ 1) * R * wpr;
        uint32_t* sXc = sX + par * R * wpr;
        const uint32_t* xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
        uint32_t* xcur = I.xbits + (size_t)par * np * wpr;
        // DetermineElite of t-1: the previous launch's elite slot, or the
        // maximum of the workgroups' keys of generation k - 1, gathered as
        // they are published (the grid barrier).  k == gens (the window's
        // variant only): the call's generations are done.
        const bool done = CONV && k == gens;
        int32_t e_prev = 0, fe_prev = 0;
        if (pending && !done) {
            unsigned long long key;
            if (k == 0) {
                key = load_dev(I.ekey + (t - 1) % 3);
            } else {
                unsigned long long sk;
                if (!gather_keys(slots + (size_t)((k - 1) & 1) * nb, nb, k - 1, abort_flag,
                                 spin_ticks, s_wkey, &s_flag, &sk))
                    return;
                key = make_key((int32_t)((uint32_t)(sk >> 32) ^ 0x80000000u),
                               (int32_t)(~(uint32_t)(sk >> 16) & 0xffffu));
            }
            e_prev = __builtin_amdgcn_readfirstlane(key_row(key));
            fe_prev = __builtin_amdgcn_readfirstlane(key_fitness(key));
            // the elite ring as the per-generation launches leave it
            if (blk == 0 && tid == 0 && k > 0) store_dev(I.ekey + (t - 1) % 3, key);
        }
        // termination test on the elite of t-1 (for k = 0 the previous
        // call's finish already made it)
        bool stop = false;
        if (CONV && pending && k > 0 && !done) {
            run = (run > 0 && fe_prev == run_fe) ? run + 1 : 1;
            run_fe = fe_prev;
            stop = run >= window;
            if (blk == 0 && tid == 0) {
                store_dev(I.conv + 8 + (int)((t - 1) & (kConvRing - 1)), fe_prev);
                if (stop) {
                    store_dev(I.conv + 1, (int32_t)(uint32_t)(uint64_t)(t - 1));
                    store_dev(I.conv + 2, (int32_t)(uint32_t)((uint64_t)(t - 1) >> 32));
                    store_dev(I.conv + 0, 1);
                }
            }
        }
        if (blk == 0 && tid == 0 && !done && !stop) store_dev(I.ekey + (t + 1) % 3, 0ull);
        // best-so-far record of t-1, written by the workgroup owning the row
        if (pending && !done && (!has_best || fe_prev > best_f)) {
            has_best = 1;
            best_f = fe_prev;
            const int re = e_prev - row0;
            if (re >= 0 && re < nrows) {
                for (int i = tid; i < wpr; i += nthr) store_dev(I.best_bits + i, sXp[re * wpr + i]);
                if (tid == 0) {
                    const int64_t tg = t - 1;
                    store_dev(I.best + 1, fe_prev);
                    store_dev(I.best + 2, sPW[((par ^ 1) * R + re) * 2]);
                    store_dev(I.best + 3, sPW[((par ^ 1) * R + re) * 2 + 1]);
                    store_dev(I.best + 4, (int32_t)(uint32_t)(uint64_t)tg);
                    store_dev(I.best + 5, (int32_t)(uint32_t)((uint64_t)tg >> 32));
                    store_dev(I.best + 6, e_prev);
                    store_dev(I.best + 0, 1);
                }
            }
        }
        if (done || stop) {
            // the planes as generation t-1 left them (its rotation pending),
            // as the per-generation launches leave them; written from one
            // place inside the loop, so the amplitude registers are neither
            // live past it nor copied for a second exit
            store_planes<K>(I, A, B, row0, r_first, ch_first, lane, first, n_items);
            break;
        }
        if (pending)
            for (int i = tid; i < wpr; i += nthr) sE[i] = load_dev(xprev + (size_t)e_prev * wpr + i);
        __syncthreads();

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
                // device scope: the elite's words are read by every workgroup
                store_dev(xcur + (size_t)c * wpr + ch * kWordsPerChunk + lane, word);
                sXc[rv * wpr + ch * kWordsPerChunk + lane] = word;
            }
            // the item tables hold nchunk * 256 entries: g0 is inside
            if (PACKED) {
                const i32x4 p4 = *reinterpret_cast<const i32x4*>(sV + g0);
                const uint32_t pw = masked_sum4(m0, m1, m2, m3, p4);
                accP += pw & 0xffffu;
                accW += pw >> 16;
            } else {
                const i32x4 v4 = *reinterpret_cast<const i32x4*>(sV + g0);
                const i32x4 w4 = *reinterpret_cast<const i32x4*>(sWt + g0);
                accP += masked_sum4(m0, m1, m2, m3, v4);
                accW += masked_sum4(m0, m1, m2, m3, w4);
            }
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
        // Evaluation closes per row; DetermineElite takes the workgroup's
        // best key (the call's last generation offers every row's key to
        // the elite slot, as the per-generation launches do)
        const bool last = k + 1 == gens;
        unsigned long long rkey = 0ull;
        if (tid < nrows) {
            const int32_t Pi = (int32_t)sSum[2 * tid], Wi = (int32_t)sSum[2 * tid + 1];
            sSum[2 * tid] = 0u;
            sSum[2 * tid + 1] = 0u;
            const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
            sF[par * R + tid] = f;
            sPW[(par * R + tid) * 2] = Pi;
            sPW[(par * R + tid) * 2 + 1] = Wi;
            const int c = row0 + tid;
            const int slot = par * np + c;
            I.fit[slot] = f;
            I.prof[slot] = Pi;
            I.wt[slot] = Wi;
            if (last) offer_key(&I.ekey[t % 3], make_key(f, c));
            rkey = slot_key(f, c);
        }
        // thread c closes row c: only the waves up to the last row hold keys
        const int nwr = (nrows + 63) >> 6;
        if (!last && wave < nwr) {
            rkey = wave_max_u64_dpp(rkey);
            if (lane == 0) s_wkey[wave] = rkey;
        }
        if (!CONV && last) {
            // the same write-back, at the end of the last generation (the
            // register allocation of the variant without the window test
            // holds the amplitudes in fewer registers this way)
            store_planes<K>(I, A, B, row0, r_first, ch_first, lane, first, n_items);
            break;
        }
        // the launch boundary ends the last generation
        if (!last) publish_key(slots + (size_t)(k & 1) * nb + blk, s_wkey, nwr, k);
    }
}

template <int K, bool CONV, bool PACKED>
__global__ __launch_bounds__(64 * kOnchipWaves) void onchip_kernel(const InstDev* __restrict__ insts,
                                                                  int R, int gens,
                                                                  int64_t spin_ticks)
{
    const InstDev I = insts[0];
    const int row0 = (int)blockIdx.x * R;
    // nrows >= 1: the grid is ceil(np / R)
    onchip_body<K, CONV, PACKED>(I, row0, min(R, I.np - row0), R, (int)blockIdx.x,
                                 (int)gridDim.x, gens, I.sync + 1, spin_ticks);
}

// Batched form: workgroup b runs tiles[b] (whole rows of one member) for
// that member's gens_arr entry (gens_all when gens_arr is NULL); the
// workgroups of one member wait only for each other.  CONV: every member of
// the launch has a convergence window; PACKED: every member's items fit the
// packed tables.
template <int K, bool CONV, bool PACKED>
__global__ __launch_bounds__(64 * kOnchipWaves) void onchip_multi_kernel(
    const InstDev* __restrict__ insts, const OnchipTile* __restrict__ tiles,
    const int32_t* __restrict__ gens_arr, int gens_all, uint32_t* abort_flag,
    int64_t spin_ticks)
{
    const OnchipTile T = tiles[blockIdx.x];
    const int gens = gens_arr ? gens_arr[T.inst] : gens_all;
    // every workgroup of the member leaves here alike
    if (gens <= 0) return;
    const InstDev I = insts[T.inst];
    onchip_body<K, CONV, PACKED>(I, T.row0, T.nrows, T.R, T.blk, T.nb, gens, abort_flag,
                                 spin_ticks);
}

// Clears the launch's abort word and, for each tile, its workgroup's key
// slots of both parities in its member's arena.
__global__ void onchip_multi_reset_kernel(const InstDev* __restrict__ insts,
                                          const OnchipTile* __restrict__ tiles, int n_tiles,
                                          uint32_t* abort_flag)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) *abort_flag = 0u;
    if (i < n_tiles) {
        const OnchipTile T = tiles[i];
        unsigned long long* slots = reinterpret_cast<unsigned long long*>(insts[T.inst].sync + 16);
        slots[T.blk] = 0ull;
        slots[T.nb + T.blk] = 0ull;
    }
}

typedef void (*OnchipFn)(const InstDev*, int, int, int64_t);

template <bool CONV, bool PACKED>
OnchipFn onchip_fn(int K)
{
    switch (K) {
        case 2: return onchip_kernel<2, CONV, PACKED>;
        case 4: return onchip_kernel<4, CONV, PACKED>;
        case 6: return onchip_kernel<6, CONV, PACKED>;
        case 8: return onchip_kernel<8, CONV, PACKED>;
        case 10: return onchip_kernel<10, CONV, PACKED>;
        default: return nullptr;
    }
}

OnchipFn onchip_fn(int K, bool conv, bool packed)
{
    if (packed) return conv ? onchip_fn<true, true>(K) : onchip_fn<false, true>(K);
    return conv ? onchip_fn<true, false>(K) : onchip_fn<false, false>(K);
}

typedef void (*OnchipMultiFn)(const InstDev*, const OnchipTile*, const int32_t*, int, uint32_t*,
                              int64_t);

template <bool CONV, bool PACKED>
OnchipMultiFn onchip_multi_fn(int K)
{
    switch (K) {
        case 2: return onchip_multi_kernel<2, CONV, PACKED>;
        case 4: return onchip_multi_kernel<4, CONV, PACKED>;
        case 6: return onchip_multi_kernel<6, CONV, PACKED>;
        case 8: return onchip_multi_kernel<8, CONV, PACKED>;
        case 10: return onchip_multi_kernel<10, CONV, PACKED>;
        default: return nullptr;
    }
}

OnchipMultiFn onchip_multi_fn(int K, bool conv, bool packed)
{
    if (packed) return conv ? onchip_multi_fn<true, true>(K) : onchip_multi_fn<false, true>(K);
    return conv ? onchip_multi_fn<true, false>(K) : onchip_multi_fn<false, false>(K);
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
        for (int cp = 0; cp < 4; ++cp) {
            const bool conv = (cp & 1) != 0, packed = (cp & 2) != 0;
            for (int K : kOnchipK) {
                const void* f = reinterpret_cast<const void*>(onchip_fn(K, conv, packed));
                int blocks = 0;
                if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)want) != hipSuccess ||
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64 * kOnchipWaves,
                                                                 want) != hipSuccess ||
                    blocks < 1) {
                    (void)hipGetLastError();
                    return;
                }
            }
        }
        lim = want;
        cus = ncu;
    });
    *lds_limit = lim;
    *n_cu = cus;
}

int64_t onchip_spin_ticks(int device, int64_t microseconds)
{
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
        khz <= 0) {
        (void)hipGetLastError();
        khz = 100000;
    }
    return (int64_t)khz * microseconds / 1000;
}

unsigned onchip_multi_variants()
{
    static std::once_flag once;
    static unsigned mask = 0;
    std::call_once(once, [] {
        size_t lim = 0;
        int ncu = 0;
        onchip_limits(&lim, &ncu);
        if (ncu == 0) return;
        for (int v = 0; v < kOnchipVariants; ++v) {
            bool ok = true;
            for (int cp = 0; cp < 4; ++cp) {
                const void* f = reinterpret_cast<const void*>(
                    onchip_multi_fn(kOnchipK[v], (cp & 1) != 0, (cp & 2) != 0));
                int blocks = 0;
                if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
                        hipSuccess ||
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64 * kOnchipWaves,
                                                                 lim) != hipSuccess ||
                    blocks < 1) {
                    (void)hipGetLastError();
                    ok = false;
                }
            }
            if (ok) mask |= 1u << v;
        }
    });
    return mask;
}

namespace {

// The on-chip launches of this library on one device run one after another,
// whatever their streams: two grids that each hold one workgroup on every
// CU could otherwise split the CUs between them and wait for each other at
// their barriers (until the bound ends both).  Each launch waits for the
// event the previous one recorded and records its own.  A stream under
// graph capture is not chained (a captured wait on an event recorded
// outside the capture is not allowed).
struct CoopChain {
    std::mutex m;
    hipEvent_t last = nullptr;
};

CoopChain& coop_chain(int device)
{
    static std::mutex mm;
    static std::map<int, CoopChain> chains;
    std::lock_guard<std::mutex> g(mm);
    return chains[device];          // std::map nodes do not move
}

// Enqueues reset() and then the cooperative launch on s, after the device's
// previous on-chip launch (see CoopChain).
template <typename Reset>
hipError_t chained_coop_launch(const void* f, unsigned blocks, void** args, size_t lds,
                               hipStream_t s, Reset reset)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(s, &cap)) != hipSuccess) return e;
    const bool chain = cap == hipStreamCaptureStatusNone;
    CoopChain& c = coop_chain(dev);
    std::lock_guard<std::mutex> g(c.m);
    if (chain) {
        if (!c.last && (e = hipEventCreateWithFlags(&c.last, hipEventDisableTiming)) != hipSuccess)
            return e;
        // an event never recorded completes at once
        if ((e = hipStreamWaitEvent(s, c.last, 0)) != hipSuccess) return e;
    }
    reset();
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipLaunchCooperativeKernel(f, dim3(blocks), dim3(64 * kOnchipWaves), args,
                                        (unsigned)lds, s)) != hipSuccess)
        return e;
    return chain ? hipEventRecord(c.last, s) : hipSuccess;
}

}  // namespace

hipError_t launch_onchip(const InstDev* dI, const OnchipPlan& p, int gens, int64_t spin_ticks,
                         hipStream_t s)
{
    if (gens <= 0) return hipSuccess;
    size_t lim = 0;
    int ncu = 0;
    onchip_limits(&lim, &ncu);
    const OnchipFn f = onchip_fn(p.K, p.conv, p.packed);
    if (!f || p.R < 1 || p.blocks < 1 || p.blocks > ncu || p.lds > lim) return hipErrorInvalidValue;
    const InstDev* a0 = dI;
    int a1 = p.R, a2 = gens;
    int64_t a3 = spin_ticks;
    void* args[] = {&a0, &a1, &a2, &a3};
    return chained_coop_launch(reinterpret_cast<const void*>(f), (unsigned)p.blocks, args, p.lds, s,
                               [&] {
                                   hipLaunchKernelGGL(onchip_reset_kernel,
                                                      dim3((unsigned)((2 * p.blocks + 255) / 256)),
                                                      dim3(256), 0, s, dI, p.blocks);
                               });
}

hipError_t launch_onchip_multi(const InstDev* dI, const OnchipTile* tiles, int n_tiles, int K,
                               bool conv, bool packed, size_t lds, const int32_t* gens_arr,
                               int gens_all, uint32_t* abort_flag, int64_t spin_ticks,
                               hipStream_t s)
{
    size_t lim = 0;
    int ncu = 0;
    onchip_limits(&lim, &ncu);
    int v = 0;
    while (v < kOnchipVariants && kOnchipK[v] != K) ++v;
    if (v == kOnchipVariants || !(onchip_multi_variants() & (1u << v)) || n_tiles < 1 ||
        n_tiles > ncu || lds > lim || !abort_flag)
        return hipErrorInvalidValue;
    const InstDev* a0 = dI;
    const OnchipTile* a1 = tiles;
    const int32_t* a2 = gens_arr;
    int a3 = gens_all;
    uint32_t* a4 = abort_flag;
    int64_t a5 = spin_ticks;
    void* args[] = {&a0, &a1, &a2, &a3, &a4, &a5};
    return chained_coop_launch(reinterpret_cast<const void*>(onchip_multi_fn(K, conv, packed)),
                               (unsigned)n_tiles, args, lds, s, [&] {
                                   hipLaunchKernelGGL(onchip_multi_reset_kernel,
                                                      dim3((unsigned)((n_tiles + 255) / 256)),
                                                      dim3(256), 0, s, dI, tiles, n_tiles,
                                                      abort_flag);
                               });
}

}  // namespace qieo
