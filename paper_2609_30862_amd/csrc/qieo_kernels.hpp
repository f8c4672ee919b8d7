// Shared declarations between the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
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
// Single-workgroup loop from global memory: rows it can hold sums for in LDS.
constexpr int kPersistentMaxRows = 2048;

// ---- host-side launchers (qieo_kernels.hip) ------------------------------
// Common conventions: gens_arr (device, one entry per instance) or, when
// NULL, gens_all gives the number of generations each instance runs in the
// current call; launch k (0-based) skips instances with gens <= k.  dI is the
// device array of instance descriptors.
hipError_t launch_init(const InstDev& I, hipStream_t s, bool f64 = false);
// Fused generation in row order: n_blocks workgroups of waves_per_block
// waves, each owning rows_per_block rows (tiles NULL: rows of instance 0 from
// blockIdx * rows_per_block).
hipError_t launch_generation(const InstDev* dI, const Tile* tiles, int n_blocks,
                             int rows_per_block, int waves_per_block, int flags, int k,
                             const int32_t* gens_arr, int gens_all, hipStream_t s);
// The same for binary64 amplitudes (instance 0 only).
hipError_t launch_generation_f64(const InstDev* dI, int n_blocks, int rows_per_block,
                                 int waves_per_block, int flags, int k, int gens_all,
                                 hipStream_t s);
// The fused generation in segment order for a single instance
// (kFlagSegments): the segment launch and the launch that closes the rows.
hipError_t launch_segments(const InstDev* dI, int np, int nchunk, int flags, int k, int gens_all,
                           bool f64, hipStream_t s);
// The same over tile tables (binary32): seg_tiles[b] = {instance, segment
// number within it}, in address order; fe_tiles[b] = {instance, first of
// the (up to) four rows the closing workgroup b takes}.
hipError_t launch_segments_tiled(const InstDev* dI, const Tile* seg_tiles, int n_seg,
                                 const Tile* fe_tiles, int n_fe, int flags, int k,
                                 const int32_t* gens_arr, hipStream_t s);
// One stage of the unfused pipeline for a single instance: kStepCip (CIP of
// generation t-1 plus the previous generation's bookkeeping), kStepQip,
// kStepFe, kStepFe | kStepDe, or kStepDe (the standalone elite reduction).
hipError_t launch_stage(const InstDev* dI, int n_blocks, int rows_per_block, int waves_per_block,
                        int stage, int k, int gens, hipStream_t s);
// Chromosome-parallel generation (one lane per chromosome), single instance.
hipError_t launch_chromosome(const InstDev* dI, int np, int k, int gens, hipStream_t s);
// Single-workgroup loops: workgroup b runs all of this call's generations of
// instance ids[b] (ids NULL: instance 0); the call's last generation's
// bookkeeping is left to launch_finish.  launch_resident keeps the whole
// state in LDS (lds_bytes = resident_lds_bytes of the largest instance, at
// most resident_lds_limit); launch_persistent works from global memory.
size_t resident_lds_bytes(int32_t np, int32_t pitch, int32_t nchunk);
// Largest dynamic LDS the resident kernel may use on the current device
// (0 if none); the first call opens the kernel up to it.
size_t resident_lds_limit();
hipError_t launch_resident(const InstDev* dI, const uint32_t* ids, int n_blocks,
                           int waves_per_block, size_t lds_bytes, const int32_t* gens_arr,
                           int gens_all, hipStream_t s);
hipError_t launch_persistent(const InstDev* dI, const uint32_t* ids, int n_blocks,
                             int waves_per_block, const int32_t* gens_arr, int gens_all,
                             hipStream_t s);
// End of a call for n_inst instances: the last generation's best-so-far
// update, the generation counter, convergence; status (may be NULL): per
// instance {generations completed, converged flag}.
hipError_t launch_finish(const InstDev* dI, int n_inst, const int32_t* gens_arr, int gens_all,
                         int64_t* status, hipStream_t s);
// Copies rows [row0, row0 + n_rows) of instance 0's state, with the pending
// rotation applied, into device buffers (any may be NULL).
hipError_t launch_export(const InstDev* dI, int row0, int n_rows, int ng,
                         void* alpha, void* beta, uint8_t* alleles,
                         int32_t* fit, int32_t* prof, int32_t* wt, bool f64, hipStream_t s);
// Best-bits words (chunk ballot layout) to plain packed bits.
hipError_t launch_bits_unpack(const uint32_t* src_words, int ng, uint32_t* dst_words,
                              hipStream_t s);

}  // namespace qieo
