// Shared declarations between the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qieo_host.hpp"
#include "qieo_layout.hpp"

namespace qieo {

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
// part_nseg: segments per row the instance's partial-sum array holds
// (hipErrorInvalidValue if the launch's segments would need more).
hipError_t launch_segments(const InstDev* dI, int np, int nchunk, int part_nseg, int flags, int k,
                           int gens_all, bool f64, hipStream_t s);
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
// On-chip loop (qieo_onchip.hip): one cooperative launch of p.blocks
// workgroups runs all gens generations of instance 0 with its planes in
// registers (p from onchip_plan); a small launch before it clears the
// abort flag and the workgroups' key slots.  The call's last generation's
// bookkeeping is left to launch_finish.  p.conv selects the variant that
// makes the convergence-window test (the other one assumes window 0).  A
// barrier wait longer than spin_ticks (device wall-clock ticks) raises the
// abort flag sync[1] and ends the launch early.
// onchip_limits: the dynamic LDS every variant may use and the CUs of the
// current device, both 0 where the loop cannot run (no cooperative launch, or
// a variant whose registers do not allow one workgroup per CU).
void onchip_limits(size_t* lds_limit, int* n_cu);
hipError_t launch_onchip(const InstDev* dI, const OnchipPlan& p, int gens, int64_t spin_ticks,
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
