// Instantiations of the objective/gradient sweep: bf16 products, plain evaluation.
#include "sweep_kernel.h"

namespace rpca {
hipError_t launch_sweep_bf16_plain(const SweepArgs& sa, bool masked, int kb, int tj, hipStream_t s) {
  return masked ? rpca_sweep::launch_tj<true, false, true>(sa, kb, tj, s)
                : rpca_sweep::launch_tj<false, false, true>(sa, kb, tj, s);
}
}  // namespace rpca
