// Instantiations of the objective/gradient sweep: f32 products, plain evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_f32_plain(const SweepArgs& sa, bool masked, int kb, int tj, hipStream_t s) {
  return masked ? rpca_sweep::launch_tj<true, false, false>(sa, kb, tj, s)
                : rpca_sweep::launch_tj<false, false, false>(sa, kb, tj, s);
}
}  // namespace rpca
