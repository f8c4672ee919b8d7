// Host-side launcher of the batched on-chip loop (qieo_onchip.hip) and the
// device queries it depends on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qieo_host.hpp"
#include "qieo_layout.hpp"

namespace qieo {

// Batched on-chip loop: one cooperative launch of n_tiles workgroups (at most
// one per CU), workgroup b running tiles[b] (device array) with the
// compiled variant K and lds bytes of dynamic LDS; member i runs gens_arr[i]
// generations (gens_all when gens_arr is NULL), its workgroups waiting only
// for each other.  conv: the variant that makes the convergence-window test
// (every member of the launch has a window); the other assumes window 0.
// packed: the variant with packed item tables (every member's items
// items_packable).
// abort_flag (device word) is cleared before the launch and raised if a
// wait runs past spin_ticks.  The call's last generation's bookkeeping is
// left to launch_finish.
hipError_t launch_onchip_multi(const InstDev* dI, const OnchipTile* tiles, int n_tiles, int K,
                               bool conv, bool packed, size_t lds, const int32_t* gens_arr,
                               int gens_all, uint32_t* abort_flag, int64_t spin_ticks,
                               hipStream_t s);
// Bound on one grid-barrier wait of the on-chip loops, in ticks of the
// device's wall clock.
int64_t onchip_spin_ticks(int device, int64_t microseconds);
// Bit v set: the batched variants kOnchipK[v] (with and without the window
// test, with and without packed item tables) fit one workgroup per CU on the current device (0 where the on-chip
// loop cannot run).
unsigned onchip_multi_variants();
}  // namespace qieo
