// Instantiations of the objective/gradient sweep with the elastic-net marginal:
// f32 products, plain and trial evaluations (the batched path and the BF16
// products use the l1 marginal only).
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_f32_elastic(const SweepArgs& sa, bool trial, bool masked, hipStream_t s) {
  using namespace rpca_sweep;
  if (masked)
    return trial ? launch_kb<true, true, false, true>(sa, s) : launch_kb<true, false, false, true>(sa, s);
  return trial ? launch_kb<false, true, false, true>(sa, s) : launch_kb<false, false, false, true>(sa, s);
}
}  // namespace rpca
