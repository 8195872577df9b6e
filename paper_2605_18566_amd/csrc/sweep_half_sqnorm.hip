// Sweep kernels instantiated for the half_sqnorm terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_half_sqnorm(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_HALF_SQNORM>(a, fresh, bf16, s, b);
}
}  // namespace hjg
