// Sweep kernels instantiated for the union-of-capture-discs terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_disc_union(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_DISC_UNION>(a, fresh, bf16, s, b);
}
}  // namespace hjg
