// Layout of a resident population and the constants shared by the HIP
// kernels, the host runtime and the host-only planning code.  Plain C++: no
// HIP header, so the planning code and its checks also build with a host
// compiler alone.
#pragma once

#include <stdint.h>

namespace qieo {

// Genes handled by one wavefront per step: 64 lanes x 4 consecutive genes,
// i.e. one Philox call (four 32-bit words) per lane.
constexpr int kChunk = 256;
// Allele words per chunk: four 64-bit lane masks (one per gene slot j of the
// lanes), stored as eight 32-bit words.
constexpr int kWordsPerChunk = 8;

// Device-side description of one resident population.  alpha and beta are
// typed float*; a binary64 instance stores doubles there (element size 8).  All arrays live in
// device memory; the struct itself is read by the kernels from a device copy.
//
// Layout (pitch = genes per row rounded up to 64, nchunk = ceil(pitch/256)):
//   alpha, beta : float[np][pitch]        SoA amplitude planes, gene-fastest
//   xbits       : uint32[2][np][nchunk*8] alleles of generation t in slot t&1;
//                 word 2j+h of chunk k holds, at bit b, gene 256k + 4(32h+b) + j
//   v, w        : int32[pitch]            item values / weights (0 in padding)
//   fit,prof,wt : int32[2][np]            eq. (1) fitness, profit, weight of t
//                                         in slot t&1
//   ekey        : uint64[3]               elite key of generation t in slot t%3:
//                 ((uint32)f ^ 0x80000000) << 32 | ~row  (max = best, lowest row)
//   best        : int32[8]                {has, f, profit, weight, gen lo, gen hi,
//                                          row, 0}
//   best_bits   : uint32[nchunk*8]        alleles of the best, in xbits layout
//   tbase       : int64[1]                number of generations completed
//   conv        : int32[64]               convergence test: [0] converged flag,
//                 [1..2] generation it converged at (lo, hi), [3] window
//                 (0 = off), [8..40) elite fitness of generation g in slot g%32
//   sync        : uint32[16] + uint64[2][min(np, kOnchipMaxBlocks)]  on-chip
//                 loop: abort flag [1], then for generations of either
//                 parity each workgroup's tagged best key (all cleared
//                 before each launch)
// Padding genes (ng <= i < pitch) hold alpha = 1, beta = 0, v = w = 0: they
// are never observed as 1 and never rotate.  Each amplitude plane is followed
// by kChunk floats of zeroed slack and v, w hold nchunk*kChunk entries, so a
// wavefront may read a whole chunk past the end of any row.
struct InstDev {
    float* alpha;
    float* beta;
    uint32_t* xbits;
    const int32_t* v;
    const int32_t* w;
    int32_t* fit;
    int32_t* prof;
    int32_t* wt;
    unsigned long long* ekey;
    int32_t* best;
    uint32_t* best_bits;
    int64_t* tbase;
    int32_t* conv;
    uint32_t* part;              // [np][nseg] (profit, weight) partial sums, segment path
    uint32_t* sync;              // on-chip loop's abort flag and workgroup keys
    int32_t np, ng, pitch, nchunk;
    int32_t capacity;
    uint32_t seed_lo, seed_hi;
};

// One work tile of a batched launch: instance index and first row.
struct Tile {
    uint32_t inst;
    uint32_t row0;
};

// Kernel variant bits ("flags"): bit 0 = prefetch the next chunk's
// amplitudes while computing the current one; bit 1 = non-temporal amplitude
// stores; bit 2 = non-temporal amplitude loads; bit 3 = re-derive the
// previous generation's alleles from beta and their draws instead of reading
// the stored words back (not in binary64 row order); bit 4 = segment
// order (single instances only): one workgroup per (row, segment of whole
// chunks), launched in address order, then a small launch that closes each
// row's partial sums into its fitness and the elite; the work shape (rows,
// waves) does not apply.  No bit changes a result.
constexpr int kFlagPrefetch = 1;
constexpr int kFlagNontemporal = 2;
constexpr int kFlagNontemporalLoads = 4;
constexpr int kFlagRecomputeAlleles = 8;
constexpr int kFlagSegments = 16;
constexpr int kFlagAll = 31;
// Segment geometry per amplitude type: 256-gene chunks per segment and waves
// per segment workgroup (each wave takes whole chunks).  The partial-sum
// array is sized for the shortest segment.
constexpr int kSegChunks32 = 4, kSegWaves32 = 4;     // binary32: 1024 genes, 4 KB a plane
constexpr int kSegChunks64 = 4, kSegWaves64 = 4;     // binary64: 1024 genes, 8 KB a plane
constexpr int kSegChunksMin = kSegChunks32 < kSegChunks64 ? kSegChunks32 : kSegChunks64;

// Steps of one generation a launch may perform.
constexpr int kStepCip = 1, kStepQip = 2, kStepFe = 4, kStepDe = 8;
constexpr int kStepAll = kStepCip | kStepQip | kStepFe | kStepDe;
// timing slots: fused generation, CIP, QIP, Evaluation, DetermineElite
constexpr int kStages = 5;
constexpr int kConvRing = 32;      // longest convergence window
// On-chip loop: most workgroups (one per CU) a launch may have.
constexpr int kOnchipMaxBlocks = 1024;
// Single-workgroup loop from global memory: rows it can hold sums for in LDS.
constexpr int kPersistentMaxRows = 2048;

// Segments of sc chunks that cover a row of nchunk chunks (the last one may
// be short).  The partial-sum array of an arena holds, per row, the count
// for the shortest segment any launch uses (kSegChunksMin); a launch whose
// segments are shorter would write past it.
constexpr int64_t seg_count(int64_t nchunk, int sc) { return (nchunk + sc - 1) / sc; }

// Launch-wide constants of the segment numbering, computed on the host so
// that no workgroup divides: the grid's split over the XCDs and, for a
// single instance, the reciprocal of its segments per row.
struct SegMap {
    int32_t xcds;        // XCDs (1: no renumbering)
    int32_t xshift;      // log2(xcds) when xcds is a power of two, else -1
    int32_t q, r;        // grid size = q * xcds + r
    int32_t nseg;        // segments per row (untiled launches)
    int32_t mshift;      // row of segment number s = (s * magic) >> mshift
    uint64_t magic;
};

// Workgroups are dispatched to the XCDs round-robin (workgroup b to XCD
// b mod xcds).  The segment number a workgroup takes gives each XCD one
// contiguous run of segment numbers: XCD x, j-th workgroup there -> the
// j-th number of run x (runs of q + 1 numbers for x < r, q after).  A
// bijection of [0, grid).  The kernels and the host checks call this same
// function.
constexpr int32_t seg_renumber(const SegMap& m, int32_t bid)
{
    if (m.xcds <= 1) return bid;
    int32_t x = 0, j = 0;
    if (m.xshift >= 0) {
        x = bid & (m.xcds - 1);
        j = bid >> m.xshift;
    } else {
        x = bid % m.xcds;
        j = bid / m.xcds;
    }
    return x * m.q + (x < m.r ? x : m.r) + j;
}

// Row of segment number s of an untiled launch: s / nseg by a multiply and
// a shift (exact for every s < 2^31; see seg_map_for).
constexpr int32_t seg_row(const SegMap& m, uint32_t s)
{
    return (int32_t)(((uint64_t)s * m.magic) >> m.mshift);
}

}  // namespace qieo
