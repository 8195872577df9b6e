// Sweep kernels instantiated for the linear terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_linear(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_LINEAR>(a, fresh, bf16, s, b);
}
}  // namespace hjg
