// Instantiations of the objective/gradient sweep: f32 products, trial evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_f32_trial(const SweepArgs& sa, bool masked, hipStream_t s) {
  return masked ? rpca_sweep::launch_kb<true, true, false>(sa, s)
                : rpca_sweep::launch_kb<false, true, false>(sa, s);
}
}  // namespace rpca
