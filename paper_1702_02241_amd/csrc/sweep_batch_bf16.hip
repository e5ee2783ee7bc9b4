// Instantiations of the batched persistent sweep (sweep_kernel.h), BF16 products.
#include "sweep_kernel.h"

namespace rpca {

hipError_t launch_sweep_batch_bf16(int kb, int tmax, const SweepArgs* args, const SweepItem* items, int nitems,
                                 unsigned* head, int grid, int lds, bool masked, bool trial, hipStream_t s) {
  using namespace rpca_sweep;
  if (masked)
    return trial ? launch_batch<true, true, true>(kb, tmax, args, items, nitems, head, grid, lds, s)
                 : launch_batch<true, false, true>(kb, tmax, args, items, nitems, head, grid, lds, s);
  return trial ? launch_batch<false, true, true>(kb, tmax, args, items, nitems, head, grid, lds, s)
               : launch_batch<false, false, true>(kb, tmax, args, items, nitems, head, grid, lds, s);
}

int sweep_batch_grid_bf16(int kb, int tmax, int lds, bool masked, bool trial) {
  using namespace rpca_sweep;
  if (masked) return trial ? batch_grid<true, true, true>(kb, tmax, lds) : batch_grid<true, false, true>(kb, tmax, lds);
  return trial ? batch_grid<false, true, true>(kb, tmax, lds) : batch_grid<false, false, true>(kb, tmax, lds);
}

}  // namespace rpca
