// Conservative safety certification: the label of every state against the
// total error budget (corollary "conservative safety certification") and the
// per-state sampling margin of the finite-sample concentration theorem.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "hjg.h"
#include "internal.h"

namespace {

constexpr int kT = 256;

int fail(int code, const std::string& msg) { return hjg_internal_fail(code, msg.c_str()); }

#define CT_HIP(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(HJG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

__global__ __launch_bounds__(kT) void zero_counts_kernel(unsigned long long* counts) {
  if (threadIdx.x < 3) counts[threadIdx.x] = 0ull;
}

// label = +1 where v > E + m, -1 where v < -(E + m), 0 otherwise (float64
// comparison); counts[label + 1] += 1.
__global__ __launch_bounds__(kT) void certify_kernel(int64_t Q, const float* v, const float* margin, double E,
                                                     int8_t* label, unsigned long long* counts) {
  __shared__ unsigned int c[3];
  if (threadIdx.x < 3) c[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (q < Q) {
    const double m = E + (margin ? (double)margin[q] : 0.0);
    const double x = (double)v[q];
    const int l = x > m ? 1 : (x < -m ? -1 : 0);
    if (label) label[q] = (int8_t)l;
    atomicAdd(&c[l + 1], 1u);
  }
  __syncthreads();
  if (counts && threadIdx.x < 3 && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

// Per-state margin at confidence delta_p: Z = exp(-c g) lies in [alpha, beta]
// (the smaller and larger of exp(-c g_min), exp(-c g_max)); with mu =
// exp(-c v), r = (beta - alpha)/mu sqrt(log(2/delta_p)/(2N)) and the margin is
// -log(1 - r)/|c| for r < 1, +inf otherwise.  In float64, in the log domain.
//
// With the effective sample sizes of the sweep, the variance-aware form of
// the empirical Bernstein inequality (two-sided, L = log(4/delta_p)):
//   rho = sqrt(2 V L / N) + 7 (beta - alpha)/mu L / (3 (N - 1)),
//   V = N/(N-1) (N/ESS - 1) the relative sample variance of the weights,
// margin = -log(1 - rho)/|c| for rho < 1.
__global__ __launch_bounds__(kT) void mc_margin_kernel(int64_t Q, const float* v, const float* c, const float* ess,
                                                       int N, double s, double L, double g_min, double g_max,
                                                       float* margin) {
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (q >= Q) return;
  const double cq = (double)c[q];
  const double a = -cq * g_min, b = -cq * g_max;      // log exp(-c g) at the two ends
  const double hi = fmax(a, b), lo = fmin(a, b);
  const double n = (double)N;
  double out;
  if (!(fabs(cq) > 0.0)) {
    out = (g_max - g_min) * s;                         // c -> 0: Hoeffding for a mean of g
  } else if (isinf(hi)) {
    out = INFINITY;
  } else {
    // (beta - alpha)/mu = exp(hi + c v) (1 - exp(lo - hi))
    const double range = exp(hi + cq * (double)v[q]) * (-expm1(lo - hi));
    double r;
    if (ess) {
      const double var = n / (n - 1.0) * fmax(n / (double)ess[q] - 1.0, 0.0);
      r = sqrt(2.0 * var * L / n) + 7.0 * range * L / (3.0 * (n - 1.0));
    } else {
      r = range * s;
    }
    out = r < 1.0 ? -log1p(-r) / fabs(cq) : INFINITY;
  }
  margin[q] = (float)out;
}

}  // namespace

extern "C" {

int hjg_certify(int64_t Q, const float* v, const float* margin, double E, int8_t* label, int64_t* counts,
                void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_certify");
  if (Q < 0 || Q > ((int64_t)1 << 40)) return fail(HJG_EINVAL, "Q must be in [0, 2^40]");
  if (!(std::isfinite(E) && E >= 0)) return fail(HJG_EINVAL, "E must be finite and >= 0");
  if (Q > 0 && !v) return fail(HJG_EINVAL, "v is required");
  if (!label && !counts) return fail(HJG_EINVAL, "label and counts are both NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts);
  if (cnt) {
    zero_counts_kernel<<<1, kT, 0, st>>>(cnt);
    CT_HIP(hipGetLastError());
  }
  if (Q == 0) return HJG_OK;
  certify_kernel<<<(unsigned)((Q + kT - 1) / kT), kT, 0, st>>>(Q, v, margin, E, label, cnt);
  CT_HIP(hipGetLastError());
  return HJG_OK;
}

int hjg_mc_margin(int64_t Q, const float* v, const float* c, const float* ess, int32_t N, double delta_p,
                  double g_min, double g_max, float* margin, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_mc_margin");
  if (Q < 0 || Q > ((int64_t)1 << 40)) return fail(HJG_EINVAL, "Q must be in [0, 2^40]");
  if (N < 1 || (ess && N < 2)) return fail(HJG_EINVAL, "N must be >= 1 (>= 2 with ess)");
  if (!(delta_p > 0 && delta_p < 1)) return fail(HJG_EINVAL, "delta_p must be in (0, 1)");
  if (!std::isfinite(g_min) || std::isnan(g_max) || !(g_max >= g_min))
    return fail(HJG_EINVAL, "need finite g_min <= g_max (g_max may be +inf)");
  if (Q == 0) return HJG_OK;
  if (!v || !c || !margin) return fail(HJG_EINVAL, "v, c and margin are required");
  const double s = std::sqrt(std::log(2.0 / delta_p) / (2.0 * (double)N));
  const double L = std::log(4.0 / delta_p);
  mc_margin_kernel<<<(unsigned)((Q + kT - 1) / kT), kT, 0, (hipStream_t)hip_stream>>>(Q, v, c, ess, N, s, L, g_min,
                                                                                         g_max, margin);
  CT_HIP(hipGetLastError());
  return HJG_OK;
}

int hjg_error_budget(const hjg_budget* b, double* E) {
  if (!b || !E) return fail(HJG_EINVAL, "NULL argument");
  if (!(b->delta_p > 0 && b->delta_p < 1) || b->N < 1 || b->K < 0 || !(b->rho >= 0) || !(b->delta >= 0) ||
      !(b->C1 >= 0) || !(b->C2 >= 0) || !(b->C3 >= 0) || !(b->eps_ql >= 0))
    return fail(HJG_EINVAL, "invalid budget terms");
  *E = b->C1 * std::pow(b->rho, (double)b->K) + b->C2 * std::sqrt(std::log(1.0 / b->delta_p) / (double)b->N) +
       b->eps_ql + b->C3 * std::sqrt(b->delta);
  return HJG_OK;
}

}  // extern "C"
