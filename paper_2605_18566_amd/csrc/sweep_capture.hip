// Sweep kernels instantiated for the capture datum of the multi-pursuer game.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_capture(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_CAPTURE>(a, fresh, bf16, s, b);
}
}  // namespace hjg
