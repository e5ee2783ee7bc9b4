// Instantiations of the batched persistent sweep (sweep_kernel.h), BF16 products.
#include "sweep_kernel.h"

namespace rpca {

hipError_t launch_sweep_batch_bf16(const SweepArgs* args, const SweepItem* items, int nitems, unsigned* head,
                                int grid, int lds, bool masked, bool trial, hipStream_t s) {
  using namespace rpca_sweep;
  if (masked)
    return trial ? launch_batch<true, true, true>(args, items, nitems, head, grid, lds, s)
                 : launch_batch<true, false, true>(args, items, nitems, head, grid, lds, s);
  return trial ? launch_batch<false, true, true>(args, items, nitems, head, grid, lds, s)
               : launch_batch<false, false, true>(args, items, nitems, head, grid, lds, s);
}

// Workgroups of the batched sweep that are resident at once (per CU x CUs).
int sweep_batch_grid_bf16(int lds, bool masked, bool trial) {
  using namespace rpca_sweep;
  int per_cu = 0;
  hipError_t e;
  if (masked)
    e = trial ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<true, true, true>, NT, lds * 4)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<true, false, true>, NT, lds * 4);
  else
    e = trial ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<false, true, true>, NT, lds * 4)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<false, false, true>, NT, lds * 4);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return per_cu * cus;
}

}  // namespace rpca
