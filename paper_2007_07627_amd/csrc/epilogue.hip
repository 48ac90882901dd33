// Weight-and-reduce pass after the closest-point search: the work
// distribution of the reduction items (the per-item arithmetic is in
// epi_item.h).
#include "epi_item.h"

namespace icp {

// single: the one-slot engine (slot 0, admitted for the whole replay), whose
// items are shared out statically by block index; otherwise items come from
// the work list's queue and are mapped to their slots.
__global__ __launch_bounds__(256) void epi_kernel(const SlotDesc* __restrict__ descs,
                                                  const SlotState* __restrict__ states,
                                                  WorkList* __restrict__ wl, int single) {
  if (single) {
    const SlotDesc& D = descs[0];
    const SlotState& S = states[0];
    if (S.status != ST_RUNNING) return;
    const bool plane = mode_plane(D.mode);
    for (int e = blockIdx.x; e < D.nepi; e += gridDim.x) {
      if (plane) epi_item<true>(D, S, e);
      else epi_item<false>(D, S, e);
    }
    return;
  }
  __shared__ int s_item;
  for (int round = 0;; ++round) {
    if (threadIdx.x == 0) s_item = queue_item(wl->q_epi, round);
    __syncthreads();
    // the item (and so the slot) is uniform over the block: kept in scalar
    // registers, the descriptor and state fields are scalar loads
    const int g = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (g >= wl->epi_total) break;
    const int lo = wave_find_slot(wl->epi_base, wl->n_active, g);
    const int slot = __builtin_amdgcn_readfirstlane(wl->slot[lo]);
    const SlotDesc& D = descs[slot];
    const SlotState& S = states[slot];
    const int e = g - wl->epi_base[lo];
    if (mode_plane(D.mode)) epi_item<true>(D, S, e);
    else epi_item<false>(D, S, e);
  }
}

void launch_epi(const SlotDesc* descs, const SlotState* states, WorkList* wl, int grid,
                bool single, hipStream_t st) {
  hipLaunchKernelGGL(epi_kernel, dim3(grid), dim3(256), 0, st, descs, states, wl, single ? 1 : 0);
}

}  // namespace icp
