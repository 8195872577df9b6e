// Sweep kernels instantiated for the min_pair_disks terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_min_pair_disks(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_MIN_PAIR_DISKS>(a, fresh, bf16, s, b);
}
}  // namespace hjg
