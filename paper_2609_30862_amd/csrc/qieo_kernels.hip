// QIEO generation kernels for gfx950 (CDNA4, wave64).
//
// One launch runs one whole generation t of every tile it is given, fused as
//     CIP(t-1)  ->  QIP(t)  ->  Evaluation(t)  ->  DetermineElite(t)
// (Sec. III-B and Fig. 1 of the paper give the order QIP, Evaluation,
// DetermineElite, CIP; the rotation of generation t-1 is deferred into the
// next launch, where it shares one read and one write of the amplitude planes
// with the observation of generation t).  The kernel boundary is the only
// grid-wide barrier a generation needs: the elite of t-1 is final when the
// launch of t starts.
//
// Work decomposition, row order (generation_kernel).  A workgroup owns R
// whole chromosomes (rows); its S wavefronts split each row into 256-gene
// chunks (wave w takes chunks w, w+S, ...), so Evaluation's gene-axis
// reduction (eq. (1)) closes inside the workgroup: DPP wave reductions, then
// LDS across the S waves, then one 64-bit atomicMax per row that can still
// win, for DetermineElite.  No cross-workgroup partial sums, no tickets, no
// memory fences.
//
// Segment order (segment_kernel + segment_fe_kernel), for populations that
// stream from HBM: one workgroup per 1024-gene segment of a row, numbered so
// that each XCD sweeps one contiguous run of segments in address order;
// segment sums are stored plainly and a second launch closes each row's
// fitness and the elite.
//
// Single-workgroup loops (resident_kernel, persistent_kernel) run all
// generations of a call for tiny populations, block barriers in place of
// launch boundaries.
//
// Per lane and chunk: 4 consecutive genes = one float4 of beta (and alpha
// when the row rotates) = one Philox4x32-10 call.  The observed alleles of a
// chunk are the four wave ballots of the comparisons: they are stored as
// eight 32-bit words and re-read as wave-uniform lane masks, so CIP's
// per-gene tests (own allele vs elite allele, target) are scalar mask logic
// and v_cndmask selects.
#include <algorithm>
#include <atomic>
#include <mutex>

#include "qieo_device.hpp"
#include "qieo_elite.hpp"
#include "qieo_host.hpp"
#include "qieo_kernels.hpp"

namespace qieo {

namespace {

// Wave sums and maxima stay in registers (DPP lane moves); the result is
// wave-uniform.  Integer sums do not depend on the order of combination.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_sum_dpp(v); }

// Opens generation t of instance I for one workgroup.  Termination test
// (convergence window): decided by every workgroup from values earlier
// launches wrote, so all of them agree; generation t-1 completes convergence
// when its elite fitness equals that of the window-1 generations before it,
// and then generation t is not run.  The instance's first workgroup (first)
// also closes the previous generation's bookkeeping: best-so-far record,
// elite fitness history, convergence flags, and the cleared elite slot of
// t+1.  Returns false when generation t is not to run.
__device__ __forceinline__ bool open_generation(const InstDev& I, int64_t t, int window,
                                                bool first, int wave, int lane, int32_t e_prev,
                                                int32_t fe_prev, const uint32_t* xprev)
{
    const bool pending = t > 0;
    bool stop = false;
    if (window > 0) {
        if (sload(I.conv) != 0) return false;       // converged in an earlier launch
        if (pending && t >= window) {
            stop = true;
            for (int j = 1; j < window; ++j)
                stop = stop && sload(I.conv + 8 + (int)((t - 1 - j) & (kConvRing - 1))) == fe_prev;
        }
    }
    if (first && wave == 0) {
        if (pending) best_update(I, t - 1, e_prev, fe_prev, xprev, lane);
        if (lane == 0) {
            if (window > 0 && pending) I.conv[8 + (int)((t - 1) & (kConvRing - 1))] = fe_prev;
            if (stop) {
                I.conv[1] = (int32_t)(uint32_t)(uint64_t)(t - 1);
                I.conv[2] = (int32_t)(uint32_t)((uint64_t)(t - 1) >> 32);
                I.conv[0] = 1;
            } else {
                I.ekey[(t + 1) % 3] = 0ull;
            }
        }
    }
    return !stop;
}

}  // namespace

// ---------------------------------------------------------------------------
// Initial state: every real gene (alpha, beta) = (1/sqrt2, 1/sqrt2); padding
// genes (1, 0).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void init_kernel(InstDev I)
{
    const size_t n = (size_t)I.np * I.pitch;
    T* alpha = reinterpret_cast<T*>(I.alpha);
    T* beta = reinterpret_cast<T*>(I.beta);
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(k % (size_t)I.pitch);
        const bool real = g < I.ng;
        alpha[k] = real ? Gate<T>::a0 : (T)1;
        beta[k] = real ? Gate<T>::a0 : (T)0;
    }
}

// ---------------------------------------------------------------------------
// The fused generation.  k is this launch's offset inside the current call:
// the generation index is t = *tbase + k, and an instance whose call asked
// for fewer than k+1 generations skips the launch.
// ---------------------------------------------------------------------------
// MODE selects the steps one launch performs (kStepAll = the fused
// generation); the unfused pipeline runs kStepCip, kStepQip and kStepFe as
// three launches, then DetermineElite by de_kernel or on the host.  FL is a
// set of kFlag* bits; none of them changes a result.
// Waves per SIMD the compiler must leave room for (register budget): with
// one binary32 row per workgroup of 8 waves, 8 per SIMD put all 32 waves of
// four workgroups on a CU at once, so 1024 rows run in one round on 256 CUs
// (at 7, a quarter of the workgroups waited for a second round).  Wider
// tiles keep the compiler's own budget (a tighter one spills registers).
template <typename T, int R>
constexpr int kRowWavesPerSimd = sizeof(T) == 4 && R == 1 ? 8 : 1;

template <typename T, int R, int FL, int MODE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kRowWavesPerSimd<T, R>))) void
generation_kernel(const InstDev* __restrict__ insts,
                                                         const Tile* __restrict__ tiles, int k,
                                                         const int32_t* __restrict__ gens_arr,
                                                         int gens_all)
{
    constexpr bool PF = (FL & kFlagPrefetch) != 0, NT = (FL & kFlagNontemporal) != 0;
    constexpr bool NTL = (FL & kFlagNontemporalLoads) != 0;
    // the fused generation may re-derive the previous alleles instead of
    // reading them back (the unfused slices always read them)
    constexpr bool RC = (FL & kFlagRecomputeAlleles) != 0 && MODE == kStepAll;
    uint32_t inst = 0, row0;
    if (tiles != nullptr) {
        const Tile tt = tiles[blockIdx.x];
        inst = tt.inst;
        row0 = tt.row0;
    } else {
        row0 = blockIdx.x * R;
    }
    const InstDev I = insts[inst];
    const int gens = gens_arr ? sload(gens_arr + inst) : gens_all;
    if (k >= gens) return;

    // Values this launch reads but never writes go through the scalar path:
    // the generation counter, the elite key of t-1 and the fitness of t-1.
    const int64_t t = sload(I.tbase) + k;
    const int par = (int)(t & 1);
    const int np = I.np;
    const int nchunk = I.nchunk;
    const int wpr = nchunk * kWordsPerChunk;
    const uint32_t* __restrict__ xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
    uint32_t* __restrict__ xcur = I.xbits + (size_t)par * np * wpr;

    const int lane = threadIdx.x & 63;
    // wave index is uniform across the wavefront; say so to the compiler so the
    // chunk loop, its addresses and its allele-mask loads stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int S = blockDim.x >> 6;

    const bool pending = t > 0;
    int32_t e_prev = 0, fe_prev = 0;
    if (pending) {
        const unsigned long long key = sload(I.ekey + (t - 1) % 3);
        e_prev = key_row(key);
        fe_prev = key_fitness(key);
    }

    constexpr bool kCip = (MODE & kStepCip) != 0, kQip = (MODE & kStepQip) != 0;
    constexpr bool kFe = (MODE & kStepFe) != 0, kDe = (MODE & kStepDe) != 0;
    const int window = MODE == kStepAll ? sload(I.conv + 3) : 0;
    if (!open_generation(I, t, window, kCip && row0 == 0, wave, lane, e_prev, fe_prev, xprev))
        return;

    const int nrows = min(R, np - (int)row0);
    typedef typename Vec4<T>::type V4;
    bool rot[R];
    const V4* arow[R];
    const V4* brow4[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rot[r] = kCip && pending && r < nrows && sload(I.fit + (par ^ 1) * np + row0 + r) < fe_prev;
        const size_t base = (size_t)(row0 + (r < nrows ? r : 0)) * I.pitch;
        arow[r] = (const V4*)(reinterpret_cast<const T*>(I.alpha) + base);
        brow4[r] = (const V4*)(reinterpret_cast<const T*>(I.beta) + base);
    }

    uint32_t accP[R], accW[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { accP[r] = 0u; accW[r] = 0u; }

    const uint32_t* __restrict__ brow = xprev + (size_t)e_prev * wpr;

    // Amplitudes of one chunk for the workgroup's rows: beta always (QIP),
    // alpha only for rows that rotate (CIP).  Lanes past the row end (only in
    // a row's last chunk) read the slack after the plane or the next row;
    // their alleles are masked to 0 and their stores skipped.
    V4 nb[R], na[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { nb[r] = V4{}; na[r] = V4{}; }
    auto load_chunk = [&](int chx) {
        const uint32_t qx = (uint32_t)chx * (kChunk / 4) + lane;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r < nrows) {
                if (NTL) {
                    if (kQip || rot[r]) nb[r] = gload_nt(brow4[r], qx);
                    if (rot[r]) na[r] = gload_nt(arow[r], qx);
                } else {
                    if (kQip || rot[r]) nb[r] = gload(brow4[r], qx);
                    if (rot[r]) na[r] = gload(arow[r], qx);
                }
            }
        }
    };
    if (PF && wave < nchunk) load_chunk(wave);

    for (int ch = wave; ch < nchunk; ch += S) {
        const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * lane;
        // lanes inside the row (all but part of a row's last chunk)
        const uint64_t actm = ballot(g0 < (uint32_t)I.pitch);
        const uint32_t q = g0 >> 2;          // float4 / int4 index in a row
        V4 cb[R], ca[R];
        if (PF) {
#pragma unroll
            for (int r = 0; r < R; ++r) { cb[r] = nb[r]; ca[r] = na[r]; }
            if (ch + S < nchunk) load_chunk(ch + S);   // next chunk in flight during this one
        } else {
            load_chunk(ch);
#pragma unroll
            for (int r = 0; r < R; ++r) { cb[r] = nb[r]; ca[r] = na[r]; }
        }
        i32x4 v4 = {0, 0, 0, 0}, w4 = {0, 0, 0, 0};
        if (kFe) {
            v4 = gload((const i32x4*)I.v, q);
            w4 = gload((const i32x4*)I.w, q);
        }
        // the elite's alleles of t-1 (at generation 0, nothing rotates and
        // the words read are the zeroed slot)
        uint64_t bm0 = 0, bm1 = 0, bm2 = 0, bm3 = 0;
        if (kCip) {
            const uint64_t* bw = reinterpret_cast<const uint64_t*>(brow + ch * kWordsPerChunk);
            bm0 = load_mask(bw); bm1 = load_mask(bw + 1);
            bm2 = load_mask(bw + 2); bm3 = load_mask(bw + 3);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nrows) break;
            const int c = (int)row0 + r;
            V4 b4 = cb[r];
            V4 a4 = ca[r];
            // the row's stored alleles of t-1 (scalar loads, in flight while
            // the draws below are computed; read for every row, so that the
            // chunk's arithmetic is one straight run of code)
            uint64_t xm[4] = {0, 0, 0, 0};
            if (kCip && !RC) {
                const uint64_t* xw = reinterpret_cast<const uint64_t*>(
                    xprev + (size_t)c * wpr + ch * kWordsPerChunk);
#pragma unroll
                for (int j = 0; j < 4; ++j) xm[j] = load_mask(xw + j);
            }
            // the draws of generation t depend on no loaded value
            Draw4 d{0u, 0u, 0u, 0u};
            if (kQip) {
                d = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
                pin_draws(d);
            }
            if (kCip) {
                if (RC) {
                    // The stored beta is the one generation t-1 observed (its
                    // rotation is still pending), so the same draw against it
                    // gives back the alleles of t-1 bit for bit.
                    const Draw4 dp = philox4x32_10(q, (uint32_t)c, (uint32_t)(t - 1), 0u,
                                                   I.seed_lo, I.seed_hi);
                    xm[0] = ballot(observe(dp.r0, b4.x)) & actm;
                    xm[1] = ballot(observe(dp.r1, b4.y)) & actm;
                    xm[2] = ballot(observe(dp.r2, b4.z)) & actm;
                    xm[3] = ballot(observe(dp.r3, b4.w)) & actm;
                }
                // genes that move: the row scores below the elite and the
                // allele differs from the elite's
                const uint64_t rowm = rot[r] ? ~0ull : 0ull;
                const uint64_t tg[4] = {bm0, bm1, bm2, bm3};
                const uint64_t mv[4] = {(xm[0] ^ bm0) & rowm, (xm[1] ^ bm1) & rowm,
                                        (xm[2] ^ bm2) & rowm, (xm[3] ^ bm3) & rowm};
                cip_chunk<V4, T>(a4, b4, mv, tg);
            }
            uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
            if (kQip) {
                m0 = ballot(observe(d.r0, b4.x)) & actm;
                m1 = ballot(observe(d.r1, b4.y)) & actm;
                m2 = ballot(observe(d.r2, b4.z)) & actm;
                m3 = ballot(observe(d.r3, b4.w)) & actm;
                store_chunk_words(xcur + (size_t)c * wpr + ch * kWordsPerChunk, m0, m1, m2, m3,
                                  lane);
            } else if (kFe) {
                // Evaluation alone: alleles of this generation from the words
                // the QIP launch stored
                const uint64_t* xw =
                    reinterpret_cast<const uint64_t*>(xcur + (size_t)c * wpr + ch * kWordsPerChunk);
                m0 = load_mask(xw); m1 = load_mask(xw + 1);
                m2 = load_mask(xw + 2); m3 = load_mask(xw + 3);
            }
            if (kFe) {
                accP[r] += masked_sum4(m0, m1, m2, m3, v4);
                accW[r] += masked_sum4(m0, m1, m2, m3, w4);
            }
            if (rot[r] && g0 < (uint32_t)I.pitch) {
                if (NT) {
                    gstore_nt((V4*)arow[r], q, a4);
                    gstore_nt((V4*)brow4[r], q, b4);
                } else {
                    gstore((V4*)arow[r], q, a4);
                    gstore((V4*)brow4[r], q, b4);
                }
            }
        }
    }

    if (!kFe) return;
    // Evaluation: close the gene-axis sums of eq. (1) inside the workgroup.
    __shared__ uint32_t red[16][R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t p = wave_sum(accP[r]);
        const uint32_t w = wave_sum(accW[r]);
        if (lane == 0) { red[wave][r][0] = p; red[wave][r][1] = w; }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)nrows) {
        const int r = threadIdx.x;
        uint32_t P = 0u, W = 0u;
        for (int s = 0; s < S; ++s) { P += red[s][r][0]; W += red[s][r][1]; }
        const int c = (int)row0 + r;
        const int32_t Pi = (int32_t)P, Wi = (int32_t)W;
        const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
        const int slot = par * np + c;
        I.fit[slot] = f;
        I.prof[slot] = Pi;
        I.wt[slot] = Wi;
        // DetermineElite: the largest key is the largest fitness, lowest row.
        if (kDe) offer_key(&I.ekey[t % 3], make_key(f, c));
    }
}

// ---------------------------------------------------------------------------
// The fused generation in segment order (single instance; T the amplitude
// type).  Rows are cut into segments of SC chunks; segment number s (segment
// s mod nseg of row s / nseg) counts through the amplitude planes in address
// order, and each XCD takes one contiguous run of segment numbers, so the
// chip sweeps the planes in address order, eight runs at a time (workgroups
// that each walk their own rows keep thousands of distant DRAM pages open at
// once).  The SW waves take chunks w, w + SW, ... of the
// segment and issue all their loads before computing.  Per gene the work is
// the fused kernel's: CIP(t-1), QIP(t), Evaluation's sums; the segment's
// (profit, weight) sums go to part[row][seg] with plain stores, and
// segment_fe_kernel closes them into fitness and the elite once every
// segment is done (the launch boundary is the only synchronisation).
// ---------------------------------------------------------------------------
template <typename T, int FL, int SC, int SW, bool TILED>
__global__ __launch_bounds__(64 * SW) void segment_kernel(const InstDev* __restrict__ insts,
                                                          const Tile* __restrict__ tiles, int k,
                                                          const int32_t* __restrict__ gens_arr,
                                                          int gens_all, SegMap map)
{
    constexpr bool NT = (FL & kFlagNontemporal) != 0, NTL = (FL & kFlagNontemporalLoads) != 0;
    constexpr bool RC = (FL & kFlagRecomputeAlleles) != 0;
    static_assert(SC % SW == 0, "whole chunks per wave");
    // the arena's partial-sum array holds seg_count(nchunk, kSegChunksMin)
    // entries per row; shorter segments would write past its end
    static_assert(SC >= kSegChunksMin, "segments shorter than the partial-sum sizing");
    constexpr int CPW = SC / SW;                          // chunks per wave
    // Workgroups are dispatched to the XCDs round-robin (workgroup b to XCD
    // b mod xcds); renumbering them gives each XCD one contiguous run of
    // segments, which it sweeps in address order.
    const int bid = seg_renumber(map, (int32_t)blockIdx.x);
    // segment number within the instance: the workgroup number (instance 0),
    // or the tile's, whose row0 field then holds a segment number
    uint32_t inst = 0, sno = (uint32_t)bid;
    int gens = gens_all;
    if constexpr (TILED) {
        const Tile tt = tiles[bid];
        inst = tt.inst;
        sno = tt.row0;
        gens = sload(gens_arr + inst);
    }
    if (k >= gens) return;
    const InstDev I = insts[inst];
    const int np = I.np, nchunk = I.nchunk, wpr = nchunk * kWordsPerChunk;
    int nseg, c;
    if constexpr (TILED) {
        nseg = (int)seg_count(nchunk, SC);
        c = (int)sno / nseg;
    } else {
        nseg = map.nseg;
        c = seg_row(map, sno);
    }
    const int seg = (int)sno - c * nseg;
    const int64_t t = sload(I.tbase) + k;
    const int par = (int)(t & 1);
    const uint32_t* __restrict__ xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
    uint32_t* __restrict__ xcur = I.xbits + (size_t)par * np * wpr;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const bool pending = t > 0;
    int32_t e_prev = 0, fe_prev = 0;
    if (pending) {
        const unsigned long long key = sload(I.ekey + (t - 1) % 3);
        e_prev = key_row(key);
        fe_prev = key_fitness(key);
    }
    if (!open_generation(I, t, sload(I.conv + 3), sno == 0, wave, lane, e_prev, fe_prev, xprev))
        return;

    const bool rot = pending && sload(I.fit + (par ^ 1) * np + c) < fe_prev;
    typedef typename Vec4<T>::type V4;
    const V4* arow = (const V4*)(reinterpret_cast<const T*>(I.alpha) + (size_t)c * I.pitch);
    const V4* brow4 = (const V4*)(reinterpret_cast<const T*>(I.beta) + (size_t)c * I.pitch);
    const uint32_t* __restrict__ erow = xprev + (size_t)e_prev * wpr;
    const uint32_t* __restrict__ orow = xprev + (size_t)c * wpr;

    // Binary64 amplitudes move between HBM and the lanes through a per-wave
    // LDS tile, so that every load and store instruction covers 1 KB of
    // consecutive addresses (a lane's own 32 bytes would take two half-dense
    // instructions): lane l transfers genes 2l, 2l+1 and 128 + 2l, 129 + 2l
    // of the chunk and computes genes 4l .. 4l + 3.
    constexpr bool kStage = sizeof(T) == 8;
    __shared__ T stage[kStage ? SW : 1][2][kStage ? kChunk : 1];

    // every load of the wave first
    V4 a4[CPW], b4[CPW];
#pragma unroll
    for (int u = 0; u < CPW; ++u) { a4[u] = V4{}; b4[u] = V4{}; }
    f64x2 la[CPW][2], lb[CPW][2];
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
        const int ch = seg * SC + u * SW + wave;
        if (ch < nchunk) {
            if constexpr (kStage) {
                const uint32_t h0 = (uint32_t)ch * (kChunk / 2) + lane, h1 = h0 + kChunk / 4;
                const f64x2* ar = (const f64x2*)arow;
                const f64x2* br = (const f64x2*)brow4;
                lb[u][0] = NTL ? gload_nt(br, h0) : gload(br, h0);
                lb[u][1] = NTL ? gload_nt(br, h1) : gload(br, h1);
                if (rot) {
                    la[u][0] = NTL ? gload_nt(ar, h0) : gload(ar, h0);
                    la[u][1] = NTL ? gload_nt(ar, h1) : gload(ar, h1);
                }
            } else {
                const uint32_t q = (uint32_t)ch * (kChunk / 4) + lane;
                b4[u] = NTL ? gload_nt(brow4, q) : gload(brow4, q);
                if (rot) a4[u] = NTL ? gload_nt(arow, q) : gload(arow, q);
            }
        }
    }
    uint32_t accP = 0u, accW = 0u;
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
        const int ch = seg * SC + u * SW + wave;
        if (ch >= nchunk) break;
        const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * lane;
        const uint64_t actm = ballot(g0 < (uint32_t)I.pitch);
        const uint32_t q = g0 >> 2;
        // Binary32 runs the chunk as one straight run: the elite's and the
        // row's own alleles of t-1 are read whether or not the row rotates
        // (scalar loads, in flight while the draws are computed) and a
        // non-rotating row's gate masks are zero.  Binary64 is bound by its
        // amplitude traffic; there a uniform branch skips the masks and the
        // gates of a row that keeps its amplitudes.
        constexpr bool kStraight = !kStage;
        uint64_t bm[4] = {0, 0, 0, 0}, xm[4] = {0, 0, 0, 0};
        if (kStraight || rot) {
            const uint64_t* bw = reinterpret_cast<const uint64_t*>(erow + ch * kWordsPerChunk);
#pragma unroll
            for (int j = 0; j < 4; ++j) bm[j] = load_mask(bw + j);
            if (!RC) {
                const uint64_t* xw = reinterpret_cast<const uint64_t*>(orow + ch * kWordsPerChunk);
#pragma unroll
                for (int j = 0; j < 4; ++j) xm[j] = load_mask(xw + j);
            }
        }
        // Item tables (cache hits): binary32 issues them here, so that they
        // arrive during the draws; binary64 after the observation (issued
        // here, the wait for its amplitudes before the LDS staging would wait
        // for them too, and held through the chunk they cost occupancy).
        i32x4 v4 = {0, 0, 0, 0}, w4 = {0, 0, 0, 0};
        if constexpr (kStraight) {
            v4 = gload((const i32x4*)I.v, q);
            w4 = gload((const i32x4*)I.w, q);
        }
        Draw4 d;
        if constexpr (kStraight) {
            d = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
            pin_draws(d);
        }
        if constexpr (kStage) {
            T* sa = stage[wave][0];
            T* sb = stage[wave][1];
            *(f64x2*)(sb + 2 * lane) = lb[u][0];
            *(f64x2*)(sb + kChunk / 2 + 2 * lane) = lb[u][1];
            if (rot) {
                *(f64x2*)(sa + 2 * lane) = la[u][0];
                *(f64x2*)(sa + kChunk / 2 + 2 * lane) = la[u][1];
            }
            __builtin_amdgcn_wave_barrier();
            b4[u] = *(const V4*)(sb + 4 * lane);
            if (rot) a4[u] = *(const V4*)(sa + 4 * lane);
            __builtin_amdgcn_wave_barrier();
        }
        V4 bb = b4[u], aa = a4[u];
        if (kStraight || rot) {
            if (RC && pending) {
                // the stored beta is the one generation t-1 observed, so its
                // draws give back that generation's alleles bit for bit
                const Draw4 dp = philox4x32_10(q, (uint32_t)c, (uint32_t)(t - 1), 0u, I.seed_lo,
                                               I.seed_hi);
                xm[0] = ballot(observe(dp.r0, bb.x)) & actm;
                xm[1] = ballot(observe(dp.r1, bb.y)) & actm;
                xm[2] = ballot(observe(dp.r2, bb.z)) & actm;
                xm[3] = ballot(observe(dp.r3, bb.w)) & actm;
            }
            const uint64_t rowm = rot ? ~0ull : 0ull;
            const uint64_t mv[4] = {(xm[0] ^ bm[0]) & rowm, (xm[1] ^ bm[1]) & rowm,
                                    (xm[2] ^ bm[2]) & rowm, (xm[3] ^ bm[3]) & rowm};
            cip_chunk<V4, T>(aa, bb, mv, bm);
        }
        if constexpr (!kStraight)
            d = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
        const uint64_t m0 = ballot(observe(d.r0, bb.x)) & actm;
        const uint64_t m1 = ballot(observe(d.r1, bb.y)) & actm;
        const uint64_t m2 = ballot(observe(d.r2, bb.z)) & actm;
        const uint64_t m3 = ballot(observe(d.r3, bb.w)) & actm;
        store_chunk_words(xcur + (size_t)c * wpr + ch * kWordsPerChunk, m0, m1, m2, m3, lane);
        if constexpr (!kStraight) {
            v4 = gload((const i32x4*)I.v, q);
            w4 = gload((const i32x4*)I.w, q);
            asm volatile("" ::"v"(v4), "v"(w4));     // both loads in flight together
        }
        accP += masked_sum4(m0, m1, m2, m3, v4);
        accW += masked_sum4(m0, m1, m2, m3, w4);
        if constexpr (kStage) {
            if (rot) {
                T* sa = stage[wave][0];
                T* sb = stage[wave][1];
                *(V4*)(sa + 4 * lane) = aa;
                *(V4*)(sb + 4 * lane) = bb;
                __builtin_amdgcn_wave_barrier();
                const f64x2 a0 = *(const f64x2*)(sa + 2 * lane);
                const f64x2 a1 = *(const f64x2*)(sa + kChunk / 2 + 2 * lane);
                const f64x2 b0 = *(const f64x2*)(sb + 2 * lane);
                const f64x2 b1 = *(const f64x2*)(sb + kChunk / 2 + 2 * lane);
                __builtin_amdgcn_wave_barrier();
                const uint32_t h0 = (uint32_t)ch * (kChunk / 2) + lane;   // f64x2 index
                const uint32_t h1 = h0 + kChunk / 4;
                f64x2* ar = (f64x2*)arow;
                f64x2* br = (f64x2*)brow4;
                if (2 * h0 < (uint32_t)I.pitch) {
                    if (NT) { gstore_nt(ar, h0, a0); gstore_nt(br, h0, b0); }
                    else { gstore(ar, h0, a0); gstore(br, h0, b0); }
                }
                if (2 * h1 < (uint32_t)I.pitch) {
                    if (NT) { gstore_nt(ar, h1, a1); gstore_nt(br, h1, b1); }
                    else { gstore(ar, h1, a1); gstore(br, h1, b1); }
                }
            }
        } else if (rot && g0 < (uint32_t)I.pitch) {
            if (NT) {
                gstore_nt((V4*)arow, q, aa);
                gstore_nt((V4*)brow4, q, bb);
            } else {
                gstore((V4*)arow, q, aa);
                gstore((V4*)brow4, q, bb);
            }
        }
    }
    // the segment's sums of eq. (1)
    __shared__ uint32_t red[SW][2];
    const uint32_t p = wave_sum(accP), w = wave_sum(accW);
    if (lane == 0) { red[wave][0] = p; red[wave][1] = w; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t P = 0u, W = 0u;
        for (int i = 0; i < SW; ++i) { P += red[i][0]; W += red[i][1]; }
        const size_t slot = ((size_t)c * nseg + seg) * 2;
        I.part[slot] = P;
        I.part[slot + 1] = W;
    }
}

// Closes generation t of the segment path: one wave per row sums the row's
// segment partials into profit and weight, applies eq. (1) and stores the
// row's fitness slot; DetermineElite offers the workgroup's best key.
__global__ __launch_bounds__(256) void segment_fe_kernel(const InstDev* __restrict__ insts,
                                                         const Tile* __restrict__ tiles, int k,
                                                         const int32_t* __restrict__ gens_arr,
                                                         int gens_all, int seg_chunks)
{
    // the workgroup's four rows: from its number (instance 0) or its tile
    uint32_t inst = 0, row0 = blockIdx.x * (blockDim.x >> 6);
    if (tiles != nullptr) {
        const Tile tt = tiles[blockIdx.x];
        inst = tt.inst;
        row0 = tt.row0;
    }
    const int gens = gens_arr ? sload(gens_arr + inst) : gens_all;
    if (k >= gens) return;
    const InstDev I = insts[inst];
    const int64_t t = sload(I.tbase) + k;
    if (sload(I.conv + 3) > 0 && sload(I.conv) != 0) return;   // generation t did not run
    const int np = I.np;
    const int nseg = (I.nchunk + seg_chunks - 1) / seg_chunks;
    const int par = (int)(t & 1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = (int)row0 + wave;
    uint32_t P = 0u, W = 0u;
    if (c < np) {
        const uint32_t* row = I.part + (size_t)c * nseg * 2;
        for (int sg = lane; sg < nseg; sg += 64) {
            P += row[2 * sg];
            W += row[2 * sg + 1];
        }
    }
    P = wave_sum(P);
    W = wave_sum(W);
    __shared__ unsigned long long red[4];
    if (lane == 0) {
        unsigned long long key = 0ull;
        if (c < np) {
            const int32_t Pi = (int32_t)P, Wi = (int32_t)W;
            const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
            const int slot = par * np + c;
            I.fit[slot] = f;
            I.prof[slot] = Pi;
            I.wt[slot] = Wi;
            key = make_key(f, c);
        }
        red[wave] = key;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long best = red[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) best = red[i] > best ? red[i] : best;
        offer_key(&I.ekey[t % 3], best);
    }
}

// DetermineElite as a launch of its own (unfused pipeline): one workgroup
// reduces the population's keys and stores the elite key of generation t.
__global__ __launch_bounds__(1024) void de_kernel(const InstDev* __restrict__ insts, int k)
{
    const InstDev I = insts[0];
    const int64_t t = *I.tbase + k;
    const int par = (int)(t & 1);
    unsigned long long best = 0ull;
    for (int c = threadIdx.x; c < I.np; c += blockDim.x) {
        const unsigned long long key = make_key(I.fit[par * I.np + c], c);
        best = key > best ? key : best;
    }
    best = wave_max_u64_dpp(best);
    __shared__ unsigned long long red[16];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = red[w] > best ? red[w] : best;
        I.ekey[t % 3] = best;
    }
}

// ---------------------------------------------------------------------------
// Persistent single-workgroup path for small populations: one workgroup runs
// generations k = 0..gens-1 of one instance (t = *tbase + k; *tbase is left
// to finish_kernel, as for per-generation launches), with block barriers in
// place of launch boundaries.  Work items are (row, chunk) pairs spread over
// the S wavefronts; per-gene arithmetic is the fused kernel's.  Everything
// this launch itself wrote earlier (alleles, fitness, elite key, convergence
// ring) is re-read with vector loads after a barrier, never through the
// scalar cache, which does not see the launch's own stores.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t vload_mask(const uint64_t* p)
{
    return uniform_mask(*(const volatile uint64_t*)p);
}

__device__ __forceinline__ int32_t vload_i32(const int32_t* p)
{
    return __builtin_amdgcn_readfirstlane(*(const volatile int32_t*)p);
}

__global__ __launch_bounds__(1024) void persistent_kernel(const InstDev* __restrict__ insts,
                                                         const uint32_t* __restrict__ ids,
                                                         const int32_t* __restrict__ gens_arr,
                                                         int gens_all)
{
    const uint32_t inst = ids ? ids[blockIdx.x] : 0u;
    const InstDev I = insts[inst];
    const int gens = gens_arr ? gens_arr[inst] : gens_all;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int S = blockDim.x >> 6;
    const int np = I.np, nchunk = I.nchunk, wpr = nchunk * kWordsPerChunk;
    const int64_t t0 = *(const volatile int64_t*)I.tbase;
    const int window = I.conv[3];
    __shared__ uint32_t sP[kPersistentMaxRows], sW[kPersistentMaxRows];
    __shared__ unsigned long long skey[16];
    __shared__ int sstop;

    for (int k = 0; k < gens; ++k) {
        const int64_t t = t0 + k;
        const int par = (int)(t & 1);
        const uint32_t* xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
        uint32_t* xcur = I.xbits + (size_t)par * np * wpr;
        const bool pending = t > 0;
        int32_t e_prev = 0, fe_prev = 0;
        if (pending) {
            const unsigned long long key = *(const volatile unsigned long long*)(I.ekey + (t - 1) % 3);
            e_prev = __builtin_amdgcn_readfirstlane(key_row(key));
            fe_prev = __builtin_amdgcn_readfirstlane(key_fitness(key));
        }
        if (threadIdx.x == 0) {
            int stop = 0;
            if (window > 0) {
                if (I.conv[0] != 0) {
                    stop = 1;
                } else if (pending && t >= window) {
                    stop = 1;
                    for (int j = 1; j < window && stop; ++j)
                        stop = ((const volatile int32_t*)I.conv)[8 + (int)((t - 1 - j) & (kConvRing - 1))] == fe_prev;
                }
            }
            sstop = stop;
        }
        for (int c = threadIdx.x; c < np; c += blockDim.x) { sP[c] = 0u; sW[c] = 0u; }
        __syncthreads();
        const bool stop = sstop != 0;
        if (wave == 0) {
            if (pending && !(window > 0 && I.conv[0] != 0))
                best_update(I, t - 1, e_prev, fe_prev, xprev, lane);
            // leave slot t+1 clear, as a per-generation launch of t would
            if (lane == 0 && !stop) I.ekey[(t + 1) % 3] = 0ull;
            if (lane == 0 && window > 0 && pending && I.conv[0] == 0) {
                I.conv[8 + (int)((t - 1) & (kConvRing - 1))] = fe_prev;
                if (stop) {
                    I.conv[1] = (int32_t)(uint32_t)(uint64_t)(t - 1);
                    I.conv[2] = (int32_t)(uint32_t)((uint64_t)(t - 1) >> 32);
                    I.conv[0] = 1;
                }
            }
        }
        if (stop) break;

        const uint32_t* brow = xprev + (size_t)e_prev * wpr;
        for (int item = wave; item < np * nchunk; item += S) {
            const int c = item / nchunk, ch = item - c * nchunk;
            const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * lane;
            const bool act = g0 < (uint32_t)I.pitch;
            const uint32_t q = g0 >> 2;
            const bool rot = pending && vload_i32(I.fit + (par ^ 1) * np + c) < fe_prev;
            const f32x4* arow = (const f32x4*)(I.alpha + (size_t)c * I.pitch);
            const f32x4* brow4 = (const f32x4*)(I.beta + (size_t)c * I.pitch);
            f32x4 b4 = gload(brow4, q);
            f32x4 a4 = b4;
            if (rot) {
                a4 = gload(arow, q);
                const uint64_t* bw = reinterpret_cast<const uint64_t*>(brow + ch * kWordsPerChunk);
                const uint64_t* xw =
                    reinterpret_cast<const uint64_t*>(xprev + (size_t)c * wpr + ch * kWordsPerChunk);
                const uint64_t bm0 = vload_mask(bw), bm1 = vload_mask(bw + 1);
                const uint64_t bm2 = vload_mask(bw + 2), bm3 = vload_mask(bw + 3);
                const uint64_t xm0 = vload_mask(xw), xm1 = vload_mask(xw + 1);
                const uint64_t xm2 = vload_mask(xw + 2), xm3 = vload_mask(xw + 3);
                float a0 = a4.x, a1 = a4.y, a2 = a4.z, a3 = a4.w;
                float b0 = b4.x, b1 = b4.y, b2 = b4.z, b3 = b4.w;
                cip_gene(a0, b0, xm0 ^ bm0, bm0);
                cip_gene(a1, b1, xm1 ^ bm1, bm1);
                cip_gene(a2, b2, xm2 ^ bm2, bm2);
                cip_gene(a3, b3, xm3 ^ bm3, bm3);
                a4 = f32x4{a0, a1, a2, a3};
                b4 = f32x4{b0, b1, b2, b3};
            }
            const Draw4 d = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
            const bool x0 = act && observe(d.r0, b4.x);
            const bool x1 = act && observe(d.r1, b4.y);
            const bool x2 = act && observe(d.r2, b4.z);
            const bool x3 = act && observe(d.r3, b4.w);
            const uint64_t m0 = ballot(x0), m1 = ballot(x1), m2 = ballot(x2), m3 = ballot(x3);
            if (lane < kWordsPerChunk) {
                const int j = lane >> 1;
                const uint64_t mm = j == 0 ? m0 : (j == 1 ? m1 : (j == 2 ? m2 : m3));
                const uint32_t word = (lane & 1) ? (uint32_t)(mm >> 32) : (uint32_t)mm;
                gstore(xcur + (size_t)c * wpr + ch * kWordsPerChunk, (uint32_t)lane, word);
            }
            const i32x4 v4 = gload((const i32x4*)I.v, q);
            const i32x4 w4 = gload((const i32x4*)I.w, q);
            uint32_t p = (x0 ? (uint32_t)v4.x : 0u) + (x1 ? (uint32_t)v4.y : 0u) +
                         (x2 ? (uint32_t)v4.z : 0u) + (x3 ? (uint32_t)v4.w : 0u);
            uint32_t w = (x0 ? (uint32_t)w4.x : 0u) + (x1 ? (uint32_t)w4.y : 0u) +
                         (x2 ? (uint32_t)w4.z : 0u) + (x3 ? (uint32_t)w4.w : 0u);
            p = wave_sum(p);
            w = wave_sum(w);
            if (lane == 0) {
                atomicAdd(&sP[c], p);
                atomicAdd(&sW[c], w);
            }
            if (rot && act) {
                gstore((f32x4*)arow, q, a4);
                gstore((f32x4*)brow4, q, b4);
            }
        }
        __syncthreads();
        // Evaluation closes in LDS; DetermineElite is a block max of the keys
        unsigned long long best = 0ull;
        for (int c = threadIdx.x; c < np; c += blockDim.x) {
            const int32_t Pi = (int32_t)sP[c], Wi = (int32_t)sW[c];
            const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
            const int slot = par * np + c;
            I.fit[slot] = f;
            I.prof[slot] = Pi;
            I.wt[slot] = Wi;
            const unsigned long long key = make_key(f, c);
            best = key > best ? key : best;
        }
        // only the waves that closed rows hold keys
        const int nw = (min(np, (int)blockDim.x) + 63) >> 6;
        if (wave < nw) {
            best = wave_max_u64_dpp(best);
            if (lane == 0) skey[wave] = best;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < nw; ++w) best = skey[w] > best ? skey[w] : best;
            I.ekey[t % 3] = best;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LDS-resident variant of the persistent loop, for populations whose whole
// state fits in one workgroup's LDS: amplitudes, both allele slots, item
// tables, fitness slots, the best-so-far bits and the convergence ring are
// staged into LDS once, every generation of the call runs on them behind two
// workgroup barriers, and the state the per-generation launches would have
// left in global memory (planes, allele words, fitness, elite keys, best
// record, convergence ring and flags) is written once at the end.  No global
// store is issued inside the loop, so the barriers never wait on memory.
// Results are those of the per-generation launches, bit for bit.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void resident_kernel(const InstDev* __restrict__ insts,
                                                       const uint32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ gens_arr,
                                                       int gens_all)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ unsigned long long skey[16];
    __shared__ int32_t sring[kConvRing];

    const uint32_t inst = ids ? ids[blockIdx.x] : 0u;
    const InstDev I = insts[inst];
    const int gens = gens_arr ? gens_arr[inst] : gens_all;
    if (gens <= 0) return;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int S = nthr >> 6;
    const int np = I.np, pitch = I.pitch, nchunk = I.nchunk, wpr = nchunk * kWordsPerChunk;
    const int plane = np * pitch;
    const int items = np * nchunk;
    // waves that close rows (thread c closes row c, c < np): only their
    // keys enter DetermineElite's block max
    const int nw = (min(np, nthr) + 63) >> 6;

    float* sA = reinterpret_cast<float*>(lds);
    float* sB = sA + plane;
    uint32_t* sX = reinterpret_cast<uint32_t*>(sB + plane);         // [2][np][wpr] by parity
    uint32_t* sBest = sX + 2 * np * wpr;                             // [wpr] best-so-far bits
    int32_t* sV = reinterpret_cast<int32_t*>(sBest + wpr);           // [nchunk * 256]
    int32_t* sWt = sV + nchunk * kChunk;
    int32_t* sF = sWt + nchunk * kChunk;                             // [2][np] fitness
    int32_t* sPr = sF + 2 * np;                                      // [2][np] profit
    int32_t* sWw = sPr + 2 * np;                                     // [2][np] weight
    uint32_t* sP = reinterpret_cast<uint32_t*>(sWw + 2 * np);        // [2][np] sums by parity
    uint32_t* sW = sP + 2 * np;

    // stage the state in
    {
        const f32x4* ga = reinterpret_cast<const f32x4*>(I.alpha);
        const f32x4* gb = reinterpret_cast<const f32x4*>(I.beta);
        f32x4* la = reinterpret_cast<f32x4*>(sA);
        f32x4* lb = reinterpret_cast<f32x4*>(sB);
        for (int i = tid; i < plane / 4; i += nthr) { la[i] = ga[i]; lb[i] = gb[i]; }
        for (int i = tid; i < 2 * np * wpr; i += nthr) sX[i] = I.xbits[i];
        for (int i = tid; i < nchunk * kChunk; i += nthr) { sV[i] = I.v[i]; sWt[i] = I.w[i]; }
        for (int i = tid; i < 2 * np; i += nthr) {
            sF[i] = I.fit[i];
            sPr[i] = I.prof[i];
            sWw[i] = I.wt[i];
            sP[i] = 0u;
            sW[i] = 0u;
        }
        if (tid < kConvRing) sring[tid] = I.conv[8 + tid];
    }
    const int64_t t0 = *(const volatile int64_t*)I.tbase;
    const int window = I.conv[3];
    const bool conv_flag = window > 0 && I.conv[0] != 0;
    // best-so-far record, kept by every thread alike; written back if changed
    int has = I.best[0];
    int32_t bf = I.best[1], bp = 0, bw = 0, be = 0;
    int64_t bt = 0;
    bool best_changed = false;
    // elite keys of the last two generations (every thread keeps them)
    unsigned long long elite = t0 > 0 ? *(const volatile unsigned long long*)(I.ekey + (t0 - 1) % 3)
                                      : 0ull;
    unsigned long long elite_before = 0ull;
    __syncthreads();

    int64_t t = t0;
    bool stopped = false;
    for (int k = 0; k < gens; ++k, ++t) {
        const int par = (int)(t & 1);
        const uint32_t* xprev = sX + (par ^ 1) * np * wpr;
        uint32_t* xcur = sX + par * np * wpr;
        uint32_t* sPc = sP + par * np;
        uint32_t* sWc = sW + par * np;
        const bool pending = t > 0;
        const int32_t e_prev =
            pending ? min(max(__builtin_amdgcn_readfirstlane(key_row(elite)), 0), np - 1) : 0;
        const int32_t fe_prev =
            pending ? __builtin_amdgcn_readfirstlane(key_fitness(elite)) : 0;
        // the draws of the wave's first item depend on no state: start them
        // before the state-dependent work
        Draw4 d_first{0u, 0u, 0u, 0u};
        if (wave < items) {
            const int c = wave / nchunk, ch = wave - c * nchunk;
            const uint32_t q = ((uint32_t)(ch * kChunk) + 4u * lane) >> 2;
            d_first = philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u, I.seed_lo, I.seed_hi);
        }
        // termination test on the elite fitness history (every thread alike)
        bool stop = false;
        if (window > 0) {
            if (conv_flag) {
                stop = true;
            } else if (pending && t >= window) {
                stop = true;
                for (int j = 1; j < window && stop; ++j)
                    stop = sring[(int)((t - 1 - j) & (kConvRing - 1))] == fe_prev;
            }
        }
        // bookkeeping of generation t-1, as the first launch of t does it
        if (pending && !conv_flag && (!has || fe_prev > bf)) {
            for (int i = tid; i < wpr; i += nthr) sBest[i] = xprev[e_prev * wpr + i];
            const int slot = (par ^ 1) * np + e_prev;
            has = 1;
            bf = fe_prev;
            bp = sPr[slot];
            bw = sWw[slot];
            bt = t - 1;
            be = e_prev;
            best_changed = true;
        }
        if (tid == 0 && window > 0 && pending && !conv_flag)
            sring[(int)((t - 1) & (kConvRing - 1))] = fe_prev;
        if (stop) {
            stopped = true;
            break;
        }

        for (int item = wave; item < items; item += S) {
            const int c = item / nchunk, ch = item - c * nchunk;
            const uint32_t g0 = (uint32_t)(ch * kChunk) + 4u * lane;
            const bool act = g0 < (uint32_t)pitch;
            const int gi = c * pitch + (act ? (int)g0 : 0);        // inside the row
            const uint32_t q = g0 >> 2;
            const bool rot =
                pending && __builtin_amdgcn_readfirstlane(sF[(par ^ 1) * np + c]) < fe_prev;
            f32x4 b4 = *reinterpret_cast<const f32x4*>(sB + gi);
            f32x4 a4 = b4;
            if (rot) {
                a4 = *reinterpret_cast<const f32x4*>(sA + gi);
                const uint64_t* bwd =
                    reinterpret_cast<const uint64_t*>(xprev + e_prev * wpr + ch * kWordsPerChunk);
                const uint64_t* xw =
                    reinterpret_cast<const uint64_t*>(xprev + c * wpr + ch * kWordsPerChunk);
                const uint64_t bm0 = uniform_mask(bwd[0]), bm1 = uniform_mask(bwd[1]);
                const uint64_t bm2 = uniform_mask(bwd[2]), bm3 = uniform_mask(bwd[3]);
                const uint64_t xm0 = uniform_mask(xw[0]), xm1 = uniform_mask(xw[1]);
                const uint64_t xm2 = uniform_mask(xw[2]), xm3 = uniform_mask(xw[3]);
                float a0 = a4.x, a1 = a4.y, a2 = a4.z, a3 = a4.w;
                float b0 = b4.x, b1 = b4.y, b2 = b4.z, b3 = b4.w;
                cip_gene(a0, b0, xm0 ^ bm0, bm0);
                cip_gene(a1, b1, xm1 ^ bm1, bm1);
                cip_gene(a2, b2, xm2 ^ bm2, bm2);
                cip_gene(a3, b3, xm3 ^ bm3, bm3);
                a4 = f32x4{a0, a1, a2, a3};
                b4 = f32x4{b0, b1, b2, b3};
            }
            const Draw4 d = item == wave ? d_first
                                         : philox4x32_10(q, (uint32_t)c, (uint32_t)t, 0u,
                                                         I.seed_lo, I.seed_hi);
            const bool x0 = act && observe(d.r0, b4.x);
            const bool x1 = act && observe(d.r1, b4.y);
            const bool x2 = act && observe(d.r2, b4.z);
            const bool x3 = act && observe(d.r3, b4.w);
            const uint64_t m0 = ballot(x0), m1 = ballot(x1), m2 = ballot(x2), m3 = ballot(x3);
            if (lane < kWordsPerChunk) {
                const int j = lane >> 1;
                const uint64_t mm = j == 0 ? m0 : (j == 1 ? m1 : (j == 2 ? m2 : m3));
                xcur[c * wpr + ch * kWordsPerChunk + lane] =
                    (lane & 1) ? (uint32_t)(mm >> 32) : (uint32_t)mm;
            }
            const int vi = act ? (int)g0 : 0;
            const i32x4 v4 = *reinterpret_cast<const i32x4*>(sV + vi);
            const i32x4 w4 = *reinterpret_cast<const i32x4*>(sWt + vi);
            const uint32_t p = (x0 ? (uint32_t)v4.x : 0u) + (x1 ? (uint32_t)v4.y : 0u) +
                               (x2 ? (uint32_t)v4.z : 0u) + (x3 ? (uint32_t)v4.w : 0u);
            const uint32_t w = (x0 ? (uint32_t)w4.x : 0u) + (x1 ? (uint32_t)w4.y : 0u) +
                               (x2 ? (uint32_t)w4.z : 0u) + (x3 ? (uint32_t)w4.w : 0u);
            const uint32_t ps = wave_sum(p);
            const uint32_t ws = wave_sum(w);
            if (lane == 0) {
                if (nchunk == 1) {              // the wave owns the row's only chunk
                    sPc[c] = ps;
                    sWc[c] = ws;
                } else {
                    atomicAdd(&sPc[c], ps);
                    atomicAdd(&sWc[c], ws);
                }
            }
            if (rot && act) {
                *reinterpret_cast<f32x4*>(sA + gi) = a4;
                *reinterpret_cast<f32x4*>(sB + gi) = b4;
            }
        }
        __syncthreads();
        // Evaluation closes in LDS (and clears this parity's sums for t+2);
        // DetermineElite is a block max of the keys
        unsigned long long best = 0ull;
        for (int c = tid; c < np; c += nthr) {
            const int32_t Pi = (int32_t)sPc[c], Wi = (int32_t)sWc[c];
            sPc[c] = 0u;
            sWc[c] = 0u;
            const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
            const int slot = par * np + c;
            sF[slot] = f;
            sPr[slot] = Pi;
            sWw[slot] = Wi;
            const unsigned long long key = make_key(f, c);
            best = key > best ? key : best;
        }
        if (wave < nw) {
            best = wave_max_u64_dpp(best);
            if (lane == 0) skey[wave] = best;
        }
        __syncthreads();
        elite_before = elite;
        elite = skey[0];
        for (int w = 1; w < nw; ++w) elite = skey[w] > elite ? skey[w] : elite;
    }
    __syncthreads();

    // write the state back: what the per-generation launches of generations
    // t0 .. t_end-1 (and, after a stop, the stopping launch) leave behind
    const int64_t t_end = t;                        // generations completed: t_end - t0
    {
        f32x4* ga = reinterpret_cast<f32x4*>(I.alpha);
        f32x4* gb = reinterpret_cast<f32x4*>(I.beta);
        const f32x4* la = reinterpret_cast<const f32x4*>(sA);
        const f32x4* lb = reinterpret_cast<const f32x4*>(sB);
        for (int i = tid; i < plane / 4; i += nthr) { ga[i] = la[i]; gb[i] = lb[i]; }
        for (int i = tid; i < 2 * np * wpr; i += nthr) I.xbits[i] = sX[i];
        for (int i = tid; i < 2 * np; i += nthr) {
            I.fit[i] = sF[i];
            I.prof[i] = sPr[i];
            I.wt[i] = sWw[i];
        }
        if (best_changed) {
            for (int i = tid; i < wpr; i += nthr) I.best_bits[i] = sBest[i];
            if (tid == 0) {
                I.best[1] = bf;
                I.best[2] = bp;
                I.best[3] = bw;
                I.best[4] = (int32_t)(uint32_t)(uint64_t)bt;
                I.best[5] = (int32_t)(uint32_t)((uint64_t)bt >> 32);
                I.best[6] = be;
                I.best[0] = 1;
            }
        }
        if (window > 0 && tid < kConvRing) I.conv[8 + tid] = sring[tid];
        if (tid == 0) {
            if (stopped && !conv_flag) {
                I.conv[1] = (int32_t)(uint32_t)(uint64_t)(t_end - 1);
                I.conv[2] = (int32_t)(uint32_t)((uint64_t)(t_end - 1) >> 32);
                I.conv[0] = 1;
            }
            if (t_end > t0) {
                I.ekey[(t_end - 1) % 3] = elite;
                I.ekey[t_end % 3] = 0ull;
                if (t_end - 2 >= t0) I.ekey[(t_end - 2) % 3] = elite_before;
            }
        }
    }
}

size_t resident_lds_limit()
{
    static std::once_flag once;
    static size_t usable = 0;
    std::call_once(once, [] {
        constexpr size_t kStatic = 1024;          // the kernel's own __shared__ variables
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess ||
            (size_t)v <= kStatic) {
            (void)hipGetLastError();
            return;
        }
        const size_t want = (size_t)v - kStatic;
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&resident_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) ==
            hipSuccess) {
            usable = want;
        } else {
            (void)hipGetLastError();
            usable = std::min<size_t>(want, 65536 - kStatic);
        }
    });
    return usable;
}

hipError_t launch_resident(const InstDev* dI, const uint32_t* ids, int n_blocks,
                           int waves_per_block, size_t lds_bytes, const int32_t* gens_arr,
                           int gens_all, hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    if (waves_per_block < 1 || waves_per_block > 16 || lds_bytes == 0 ||
        lds_bytes > resident_lds_limit())
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(resident_kernel, dim3((unsigned)n_blocks),
                       dim3((unsigned)(64 * waves_per_block)), lds_bytes, s, dI, ids, gens_arr,
                       gens_all);
    return hipGetLastError();
}

hipError_t launch_persistent(const InstDev* dI, const uint32_t* ids, int n_blocks,
                             int waves_per_block, const int32_t* gens_arr, int gens_all,
                             hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    if (waves_per_block < 1 || waves_per_block > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(persistent_kernel, dim3((unsigned)n_blocks),
                       dim3((unsigned)(64 * waves_per_block)), 0, s, dI, ids, gens_arr, gens_all);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Chromosome-parallel mapping (eq. (3) of the paper): one lane per
// chromosome walks that chromosome's genes serially, doing CIP(t-1), QIP,
// Evaluation and the elite atomicMax of generation t.  Neighbouring lanes
// touch addresses a whole row apart, so loads do not coalesce: this kernel
// exists to measure that mapping, not to be fast.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void chromosome_kernel(const InstDev* __restrict__ insts, int k,
                                                        int gens)
{
    const InstDev I = insts[0];
    if (k >= gens) return;
    const int64_t t = sload(I.tbase) + k;
    const int par = (int)(t & 1);
    const int np = I.np;
    const int wpr = I.nchunk * kWordsPerChunk;
    const uint32_t* __restrict__ xprev = I.xbits + (size_t)(par ^ 1) * np * wpr;
    uint32_t* __restrict__ xcur = I.xbits + (size_t)par * np * wpr;
    const int lane = threadIdx.x;
    const bool pending = t > 0;
    int32_t e_prev = 0, fe_prev = 0;
    if (pending) {
        const unsigned long long key = sload(I.ekey + (t - 1) % 3);
        e_prev = key_row(key);
        fe_prev = key_fitness(key);
    }
    if (blockIdx.x == 0) {
        if (pending) best_update(I, t - 1, e_prev, fe_prev, xprev, lane);
        if (lane == 0) I.ekey[(t + 1) % 3] = 0ull;
    }
    const int c = blockIdx.x * 64 + lane;
    if (c >= np) return;
    const bool rot = pending && I.fit[(par ^ 1) * np + c] < fe_prev;
    float* arow = I.alpha + (size_t)c * I.pitch;
    float* brow = I.beta + (size_t)c * I.pitch;
    const uint32_t* own = xprev + (size_t)c * wpr;
    const uint32_t* eli = xprev + (size_t)e_prev * wpr;
    uint32_t P = 0u, W = 0u;
    for (int ch = 0; ch < I.nchunk; ++ch) {
        uint32_t words[kWordsPerChunk];
        for (int w = 0; w < kWordsPerChunk; ++w) words[w] = 0u;
        for (int L = 0; L < 64; ++L) {
            const int g0 = ch * kChunk + 4 * L;
            if (g0 >= I.pitch) break;
            float a[4], b[4];
            for (int j = 0; j < 4; ++j) {
                a[j] = arow[g0 + j];
                b[j] = brow[g0 + j];
            }
            const int wsel = L >> 5, bit = L & 31;
            if (rot) {
                for (int j = 0; j < 4; ++j) {
                    const int wi = ch * kWordsPerChunk + 2 * j + wsel;
                    const bool xo = (own[wi] >> bit) & 1u;
                    const bool be = (eli[wi] >> bit) & 1u;
                    if (xo != be) cip_gene_lane(a[j], b[j], be);
                }
            }
            const Draw4 d = philox4x32_10((uint32_t)(g0 >> 2), (uint32_t)c, (uint32_t)t, 0u,
                                          I.seed_lo, I.seed_hi);
            const uint32_t r4[4] = {d.r0, d.r1, d.r2, d.r3};
            for (int j = 0; j < 4; ++j) {
                const bool x = g0 + j < I.ng && observe(r4[j], b[j]);
                if (x) {
                    words[2 * j + wsel] |= 1u << bit;
                    P += (uint32_t)I.v[g0 + j];
                    W += (uint32_t)I.w[g0 + j];
                }
                if (rot) {
                    arow[g0 + j] = a[j];
                    brow[g0 + j] = b[j];
                }
            }
        }
        for (int w = 0; w < kWordsPerChunk; ++w)
            xcur[(size_t)c * wpr + ch * kWordsPerChunk + w] = words[w];
    }
    const int32_t Pi = (int32_t)P, Wi = (int32_t)W;
    const int32_t f = (Wi <= I.capacity) ? Pi : -(Wi - I.capacity);
    const int slot = par * np + c;
    I.fit[slot] = f;
    I.prof[slot] = Pi;
    I.wt[slot] = Wi;
    offer_key(&I.ekey[t % 3], make_key(f, c));
}

hipError_t launch_chromosome(const InstDev* dI, int np, int k, int gens, hipStream_t s)
{
    hipLaunchKernelGGL(chromosome_kernel, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, s, dI, k,
                       gens);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// End of a call: best-so-far update for the last generation of the call and
// advance of the generation counter.  One workgroup (one wave) per instance.
// ---------------------------------------------------------------------------
__global__ void finish_kernel(const InstDev* __restrict__ insts,
                              const int32_t* __restrict__ gens_arr, int gens_all,
                              int64_t* __restrict__ status)
{
    const InstDev I = insts[blockIdx.x];
    const int gens = gens_arr ? gens_arr[blockIdx.x] : gens_all;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x >= 64) return;
    int64_t done = *I.tbase;
    const int window = I.conv[3];
    int converged = window > 0 ? I.conv[0] : 0;
    if (gens > 0) {
        if (converged) {
            // a launch of this call (or of an earlier one) found convergence
            done = (int64_t)(((uint64_t)(uint32_t)I.conv[2] << 32) | (uint32_t)I.conv[1]) + 1;
        } else {
            const int64_t tl = done + gens - 1;
            const unsigned long long key = I.ekey[tl % 3];
            const int32_t fe = key_fitness(key);
            const uint32_t* xg = I.xbits + (size_t)(tl & 1) * I.np * I.nchunk * kWordsPerChunk;
            best_update(I, tl, key_row(key), fe, xg, lane);
            if (window > 0 && lane == 0) {
                I.conv[8 + (int)(tl & (kConvRing - 1))] = fe;
                bool stop = tl + 1 >= window;
                for (int j = 1; j < window && stop; ++j)
                    stop = I.conv[8 + (int)((tl - j) & (kConvRing - 1))] == fe;
                if (stop) {
                    I.conv[1] = (int32_t)(uint32_t)(uint64_t)tl;
                    I.conv[2] = (int32_t)(uint32_t)((uint64_t)tl >> 32);
                    I.conv[0] = 1;
                    converged = 1;
                }
            }
            done = tl + 1;
        }
        if (lane == 0) *I.tbase = done;
    }
    if (status && lane == 0) {
        status[2 * blockIdx.x] = done;
        status[2 * blockIdx.x + 1] = converged;
    }
}

// ---------------------------------------------------------------------------
// Export of rows [row0, row0+n) after the last completed generation t-1:
// amplitudes with CIP(t-1) applied (state untouched), alleles and fitness of
// t-1.  Block = 256 threads = 4 waves, one gene per thread.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void export_kernel(const InstDev* __restrict__ insts, int row0, T* alpha, T* beta,
                              uint8_t* alleles)
{
    const InstDev I = insts[0];
    const int64_t t = *I.tbase;
    const int c = row0 + blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = g < I.ng;
    const int wpr = I.nchunk * kWordsPerChunk;
    const size_t src = (size_t)c * I.pitch + (act ? g : 0);
    T a = act ? reinterpret_cast<const T*>(I.alpha)[src] : (T)1;
    T b = act ? reinterpret_cast<const T*>(I.beta)[src] : (T)0;
    bool x = false, bel = false, rot = false;
    if (t > 0 && act) {
        const int par = (int)((t - 1) & 1);
        const uint32_t* xg = I.xbits + (size_t)par * I.np * wpr;
        const unsigned long long key = I.ekey[(t - 1) % 3];
        const int e = key_row(key);
        const int32_t fe = key_fitness(key);
        const int ch = g / kChunk, q = g % kChunk, L = q >> 2, j = q & 3;
        const int word = ch * kWordsPerChunk + 2 * j + (L >> 5);
        const int bit = L & 31;
        x = (xg[(size_t)c * wpr + word] >> bit) & 1u;
        bel = (xg[(size_t)e * wpr + word] >> bit) & 1u;
        rot = (I.fit[par * I.np + c] < fe) && (x != bel);
    }
    const uint64_t rm = ballot(rot), tm = ballot(bel);
    cip_gene(a, b, rm, tm);
    if (act) {
        const size_t dst = (size_t)blockIdx.y * I.ng + g;
        if (alpha) alpha[dst] = a;
        if (beta) beta[dst] = b;
        if (alleles) alleles[dst] = x ? 1 : 0;
    }
}

__global__ void export_rows_kernel(const InstDev* __restrict__ insts, int row0, int n_rows,
                                   int32_t* fit, int32_t* prof, int32_t* wt)
{
    const InstDev I = insts[0];
    const int64_t t = *I.tbase;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int slot = (int)((t - 1) & 1) * I.np + row0 + r;
    const bool any = t > 0;
    if (fit) fit[r] = any ? I.fit[slot] : 0;
    if (prof) prof[r] = any ? I.prof[slot] : 0;
    if (wt) wt[r] = any ? I.wt[slot] : 0;
}

// Chunked-ballot allele words -> plain packed bits (gene i = bit i%32 of word i/32).
__global__ void bits_unpack_kernel(const uint32_t* __restrict__ src, int ng, uint32_t* dst)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = (ng + 31) / 32;
    if (q >= nw) return;
    uint32_t out = 0u;
    for (int b = 0; b < 32; ++b) {
        const int g = 32 * q + b;
        if (g >= ng) break;
        const int ch = g / kChunk, r = g % kChunk, L = r >> 2, j = r & 3;
        const uint32_t w = src[ch * kWordsPerChunk + 2 * j + (L >> 5)];
        out |= ((w >> (L & 31)) & 1u) << b;
    }
    dst[q] = out;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_init(const InstDev& I, hipStream_t s, bool f64)
{
    const size_t n = (size_t)I.np * I.pitch;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (f64)
        hipLaunchKernelGGL(init_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, I);
    else
        hipLaunchKernelGGL(init_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, I);
    return hipGetLastError();
}

// XCDs of the current device (1 if the runtime cannot tell), cached per
// device.
static int xcd_count()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 1;
    }
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess ||
            n < 1) {
            (void)hipGetLastError();
            n = 1;
        }
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Segment launch and the launch closing the rows, for n_seg segment
// workgroups and n_fe row-closing workgroups (four rows each).
static hipError_t segments_common(const InstDev* dI, const Tile* seg_tiles, int64_t n_seg,
                                  int nseg_row, const Tile* fe_tiles, int64_t n_fe, int flags,
                                  int k, const int32_t* gens_arr, int gens_all, bool f64,
                                  hipStream_t s)
{
    if (n_seg <= 0 || n_fe <= 0 || n_seg > INT32_MAX) return hipErrorInvalidValue;
    if (!seg_tiles && nseg_row < 1) return hipErrorInvalidValue;
    static_assert(kFlagNontemporal == 2 && kFlagNontemporalLoads == 4 &&
                      kFlagRecomputeAlleles == 8,
                  "segment variants below are spelled out by value");
    const int sc = f64 ? kSegChunks64 : kSegChunks32;
    const int sw = f64 ? kSegWaves64 : kSegWaves32;
    const dim3 grid((unsigned)n_seg), block((unsigned)(64 * sw));
    const SegMap map = seg_map_for(n_seg, xcd_count(), seg_tiles ? 0 : nseg_row);
#define QIEO_SEG(TT, FF, SC, SW)                                                               \
    do {                                                                                       \
        if (seg_tiles)                                                                         \
            hipLaunchKernelGGL((segment_kernel<TT, FF, SC, SW, true>), grid, block, 0, s, dI,  \
                               seg_tiles, k, gens_arr, gens_all, map);                         \
        else                                                                                   \
            hipLaunchKernelGGL((segment_kernel<TT, FF, SC, SW, false>), grid, block, 0, s, dI, \
                               seg_tiles, k, gens_arr, gens_all, map);                         \
    } while (0)
#define QIEO_SEG_T(TT, SC, SW)                                                                 \
    switch (flags & (kFlagNontemporal | kFlagNontemporalLoads | kFlagRecomputeAlleles)) {      \
    case 0: QIEO_SEG(TT, 0, SC, SW); break;                                                    \
    case 2: QIEO_SEG(TT, 2, SC, SW); break;                                                    \
    case 4: QIEO_SEG(TT, 4, SC, SW); break;                                                    \
    case 6: QIEO_SEG(TT, 6, SC, SW); break;                                                    \
    case 8: QIEO_SEG(TT, 8, SC, SW); break;                                                    \
    case 10: QIEO_SEG(TT, 10, SC, SW); break;                                                  \
    case 12: QIEO_SEG(TT, 12, SC, SW); break;                                                  \
    default: QIEO_SEG(TT, 14, SC, SW); break;                                                  \
    }
    if (f64 && seg_tiles) return hipErrorInvalidValue;     // tiled launches are binary32
    if (f64) {
        QIEO_SEG_T(double, kSegChunks64, kSegWaves64)
    } else {
        QIEO_SEG_T(float, kSegChunks32, kSegWaves32)
    }
#undef QIEO_SEG_T
#undef QIEO_SEG
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(segment_fe_kernel, dim3((unsigned)n_fe), dim3(256), 0, s, dI, fe_tiles, k,
                       gens_arr, gens_all, sc);
    return hipGetLastError();
}

hipError_t launch_segments(const InstDev* dI, int np, int nchunk, int part_nseg, int flags, int k,
                           int gens_all, bool f64, hipStream_t s)
{
    if (np <= 0) return hipErrorInvalidValue;
    const int sc = f64 ? kSegChunks64 : kSegChunks32;
    const int64_t nseg = seg_count(nchunk, sc);
    // each segment stores its sums at part[row][segment]: never more
    // segments per row than the arena's partial-sum array holds
    if (nseg > part_nseg) return hipErrorInvalidValue;
    return segments_common(dI, nullptr, (int64_t)np * nseg, (int)nseg, nullptr, (np + 3) / 4,
                           flags, k, nullptr, gens_all, f64, s);
}

hipError_t launch_segments_tiled(const InstDev* dI, const Tile* seg_tiles, int n_seg,
                                 const Tile* fe_tiles, int n_fe, int flags, int k,
                                 const int32_t* gens_arr, hipStream_t s)
{
    return segments_common(dI, seg_tiles, n_seg, 0, fe_tiles, n_fe, flags, k, gens_arr, 0, false,
                           s);
}

hipError_t launch_generation(const InstDev* dI, const Tile* tiles, int n_blocks,
                             int rows_per_block, int waves_per_block, int flags, int k,
                             const int32_t* gens_arr, int gens_all, hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    if (flags & kFlagSegments) return hipErrorInvalidValue;    // launch_segments
    if (waves_per_block < 1 || waves_per_block > 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_blocks), block((unsigned)(64 * waves_per_block));
#define QIEO_LAUNCH(RR, FF)                                                                    \
    hipLaunchKernelGGL((generation_kernel<float, RR, FF, kStepAll>), grid, block, 0, s, dI,    \
                       tiles, k, gens_arr, gens_all)
#define QIEO_LAUNCH_R(RR)                                                                      \
    switch (flags & 15) {                                                                      \
    case 0: QIEO_LAUNCH(RR, 0); break;                                                         \
    case 1: QIEO_LAUNCH(RR, 1); break;                                                         \
    case 2: QIEO_LAUNCH(RR, 2); break;                                                         \
    case 3: QIEO_LAUNCH(RR, 3); break;                                                         \
    case 4: QIEO_LAUNCH(RR, 4); break;                                                         \
    case 5: QIEO_LAUNCH(RR, 5); break;                                                         \
    case 6: QIEO_LAUNCH(RR, 6); break;                                                         \
    case 7: QIEO_LAUNCH(RR, 7); break;                                                         \
    case 8: QIEO_LAUNCH(RR, 8); break;                                                         \
    case 9: QIEO_LAUNCH(RR, 9); break;                                                         \
    case 10: QIEO_LAUNCH(RR, 10); break;                                                       \
    case 11: QIEO_LAUNCH(RR, 11); break;                                                       \
    case 12: QIEO_LAUNCH(RR, 12); break;                                                       \
    case 13: QIEO_LAUNCH(RR, 13); break;                                                       \
    case 14: QIEO_LAUNCH(RR, 14); break;                                                       \
    default: QIEO_LAUNCH(RR, 15); break;                                                       \
    }
    switch (rows_per_block) {
    case 1: QIEO_LAUNCH_R(1); break;
    case 2: QIEO_LAUNCH_R(2); break;
    case 4: QIEO_LAUNCH_R(4); break;
    default: return hipErrorInvalidValue;
    }
#undef QIEO_LAUNCH_R
#undef QIEO_LAUNCH
    return hipGetLastError();
}

hipError_t launch_generation_f64(const InstDev* dI, int n_blocks, int rows_per_block,
                                 int waves_per_block, int flags, int k, int gens_all,
                                 hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    if (waves_per_block < 1 || waves_per_block > 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_blocks), block((unsigned)(64 * waves_per_block));
#define QIEO_LAUNCH(RR, FF)                                                                    \
    hipLaunchKernelGGL((generation_kernel<double, RR, FF, kStepAll>), grid, block, 0, s, dI,   \
                       (const Tile*)nullptr, k, (const int32_t*)nullptr, gens_all)
#define QIEO_LAUNCH_R(RR)                                                                      \
    switch (flags & 7) {                                                                       \
    case 0: QIEO_LAUNCH(RR, 0); break;                                                         \
    case 1: QIEO_LAUNCH(RR, 1); break;                                                         \
    case 2: QIEO_LAUNCH(RR, 2); break;                                                         \
    case 3: QIEO_LAUNCH(RR, 3); break;                                                         \
    case 4: QIEO_LAUNCH(RR, 4); break;                                                         \
    case 5: QIEO_LAUNCH(RR, 5); break;                                                         \
    case 6: QIEO_LAUNCH(RR, 6); break;                                                         \
    default: QIEO_LAUNCH(RR, 7); break;                                                        \
    }
    switch (rows_per_block) {
    case 1: QIEO_LAUNCH_R(1); break;
    case 2: QIEO_LAUNCH_R(2); break;
    case 4: QIEO_LAUNCH_R(4); break;
    default: return hipErrorInvalidValue;
    }
#undef QIEO_LAUNCH_R
#undef QIEO_LAUNCH
    return hipGetLastError();
}

hipError_t launch_stage(const InstDev* dI, int n_blocks, int rows_per_block, int waves_per_block,
                        int stage, int k, int gens, hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    if (waves_per_block < 1 || waves_per_block > 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_blocks), block((unsigned)(64 * waves_per_block));
    if (stage == kStepDe) {
        hipLaunchKernelGGL(de_kernel, dim3(1), dim3(1024), 0, s, dI, k);
        return hipGetLastError();
    }
#define QIEO_STAGE(RR, MM)                                                                     \
    hipLaunchKernelGGL((generation_kernel<float, RR, kFlagNontemporal, MM>), grid, block, 0, s, \
                       dI, (const Tile*)nullptr, k, (const int32_t*)nullptr, gens)
#define QIEO_STAGE_R(RR)                                                                       \
    switch (stage) {                                                                           \
    case kStepCip: QIEO_STAGE(RR, kStepCip); break;                                            \
    case kStepQip: QIEO_STAGE(RR, kStepQip); break;                                            \
    case kStepFe: QIEO_STAGE(RR, kStepFe); break;                                              \
    case kStepFe | kStepDe: QIEO_STAGE(RR, kStepFe | kStepDe); break;                          \
    default: return hipErrorInvalidValue;                                                      \
    }
    switch (rows_per_block) {
    case 1: QIEO_STAGE_R(1); break;
    case 2: QIEO_STAGE_R(2); break;
    case 4: QIEO_STAGE_R(4); break;
    default: return hipErrorInvalidValue;
    }
#undef QIEO_STAGE_R
#undef QIEO_STAGE
    return hipGetLastError();
}

hipError_t launch_finish(const InstDev* dI, int n_inst, const int32_t* gens_arr, int gens_all,
                         int64_t* status, hipStream_t s)
{
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_kernel, dim3((unsigned)n_inst), dim3(64), 0, s, dI, gens_arr,
                       gens_all, status);
    return hipGetLastError();
}

hipError_t launch_export(const InstDev* dI, int row0, int n_rows, int ng, void* alpha,
                         void* beta, uint8_t* alleles, int32_t* fit, int32_t* prof,
                         int32_t* wt, bool f64, hipStream_t s)
{
    if (n_rows <= 0) return hipSuccess;
    if (alpha || beta || alleles) {
        const dim3 grid((unsigned)((ng + 255) / 256), (unsigned)n_rows);
        if (f64)
            hipLaunchKernelGGL(export_kernel<double>, grid, dim3(256), 0, s, dI, row0,
                               (double*)alpha, (double*)beta, alleles);
        else
            hipLaunchKernelGGL(export_kernel<float>, grid, dim3(256), 0, s, dI, row0,
                               (float*)alpha, (float*)beta, alleles);
    }
    if (fit || prof || wt)
        hipLaunchKernelGGL(export_rows_kernel, dim3((unsigned)((n_rows + 255) / 256)), dim3(256),
                           0, s, dI, row0, n_rows, fit, prof, wt);
    return hipGetLastError();
}

hipError_t launch_bits_unpack(const uint32_t* src_words, int ng, uint32_t* dst_words,
                              hipStream_t s)
{
    const int nw = (ng + 31) / 32;
    hipLaunchKernelGGL(bits_unpack_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                       src_words, ng, dst_words);
    return hipGetLastError();
}

}  // namespace qieo
