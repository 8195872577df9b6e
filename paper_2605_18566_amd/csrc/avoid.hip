// Reach-avoid tube in splitting form: after each time step the value is
// lifted onto the obstacle constraint v >= -l_A(x) of the avoid set
// A = {l_A <= 0} (the viscous reach-avoid variational inequality,
// HJI-RCBRAT-Visc), so no state of A is ever counted as reached.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "hjg.h"
#include "internal.h"
#include "kernels.h"

namespace {

constexpr int kT = 256;
constexpr unsigned kMaxBlocks = 1u << 20;   // grid-stride beyond this many blocks

int fail(int code, const std::string& msg) { return hjg_internal_fail(code, msg.c_str()); }

// One state per thread: l_A and D l_A from the datum rules of the sweep, then
// v <- max(v, -l_A) with the gradient of the winning branch.  Memory: n + 1
// floats read and (where active) n + 1 written per state, plus one flag byte.
template <int NM>
__global__ __launch_bounds__(kT) void avoid_kernel(hjg::DatumP dp, int64_t Q, const float* __restrict__ x,
                                                   float* __restrict__ v, float* __restrict__ grad,
                                                   uint8_t* __restrict__ active) {
  for (int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x; q < Q; q += (int64_t)gridDim.x * kT) {
    float xs[NM], g[NM];
#pragma unroll
    for (int d = 0; d < NM; ++d) xs[d] = d < dp.n ? x[(int64_t)d * Q + q] : 0.f;
    const float h = -hjg::datum_and_grad<NM>(dp, xs, g, q, Q);
    const bool on = h > v[q];
    if (on) {
      v[q] = h;
      if (grad) {
#pragma unroll
        for (int d = 0; d < NM; ++d)
          if (d < dp.n) grad[(int64_t)d * Q + q] = -g[d];
      }
    }
    if (active) active[q] = on ? 1 : 0;
  }
}

}  // namespace

int hjg_avoid_project(const hjg_problem* obstacle, int64_t Q, const float* x, float* v, float* grad,
                      uint8_t* active, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_avoid_project");
  int rc;
  if ((rc = hjg::detail::check_datum(obstacle))) return rc;
  if (Q < 0 || Q > ((int64_t)1 << 40)) return fail(HJG_EINVAL, "Q must be in [0, 2^40]");
  if (Q == 0) return HJG_OK;
  if (!x || !v) return fail(HJG_EINVAL, "x and v are required");
  const hjg::DatumP dp = hjg::detail::datum_params(obstacle);
  hipStream_t st = (hipStream_t)hip_stream;
  const unsigned blocks = (unsigned)std::min<int64_t>((Q + kT - 1) / kT, kMaxBlocks);
  switch (hjg::n_bucket(obstacle->n)) {
    case 4: avoid_kernel<4><<<blocks, kT, 0, st>>>(dp, Q, x, v, grad, active); break;
    case 8: avoid_kernel<8><<<blocks, kT, 0, st>>>(dp, Q, x, v, grad, active); break;
    case 16: avoid_kernel<16><<<blocks, kT, 0, st>>>(dp, Q, x, v, grad, active); break;
    case 32: avoid_kernel<32><<<blocks, kT, 0, st>>>(dp, Q, x, v, grad, active); break;
    default: avoid_kernel<48><<<blocks, kT, 0, st>>>(dp, Q, x, v, grad, active); break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HJG_EHIP, std::string("avoid_kernel: ") + hipGetErrorString(e));
  return HJG_OK;
}
