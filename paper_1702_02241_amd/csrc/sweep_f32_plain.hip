// Instantiations of the objective/gradient sweep: f32 products, plain evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_f32_plain(const SweepArgs& sa, bool masked, hipStream_t s) {
  return masked ? rpca_sweep::launch_kb<true, false, false>(sa, s)
                : rpca_sweep::launch_kb<false, false, false>(sa, s);
}
}  // namespace rpca
