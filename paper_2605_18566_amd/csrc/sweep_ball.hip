// Sweep kernels instantiated for the ball terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_ball(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_BALL>(a, fresh, bf16, s, b);
}
}  // namespace hjg
