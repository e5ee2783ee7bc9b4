// Instantiations of the objective/gradient sweep: bf16 products, plain evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_bf16_plain(const SweepArgs& sa, bool masked, hipStream_t s) {
  return masked ? rpca_sweep::launch_kb<true, false, true>(sa, s)
                : rpca_sweep::launch_kb<false, false, true>(sa, s);
}
}  // namespace rpca
