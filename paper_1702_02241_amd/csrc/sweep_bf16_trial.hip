// Instantiations of the objective/gradient sweep: bf16 products, trial evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_bf16_trial(const SweepArgs& sa, bool masked, hipStream_t s) {
  return masked ? rpca_sweep::launch_kb<true, true, true>(sa, s)
                : rpca_sweep::launch_kb<false, true, true>(sa, s);
}
}  // namespace rpca
