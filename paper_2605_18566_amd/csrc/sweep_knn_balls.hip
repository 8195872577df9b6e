// Sweep kernels instantiated for the knn_balls terminal datum.
#include "sweep_impl.h"

namespace hjg {
hipError_t launch_sweep_knn_balls(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_d<HJG_L_KNN_BALLS>(a, fresh, bf16, s, b);
}
}  // namespace hjg
