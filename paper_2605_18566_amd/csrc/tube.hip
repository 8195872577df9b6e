// Time marching with the surrogate network as the datum: the sample points of
// a query chunk become network inputs, and after the network's forward pass
// one block per query folds the value outputs into the log-sum-exp partials
// of the pair loops (log2 units, maximum-rescaled sums).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace hjg {
namespace {

__device__ __forceinline__ float table_z(const void* table, int bf16, int64_t idx) {
  if (bf16) return __uint_as_float((uint32_t)static_cast<const uint16_t*>(table)[idx] << 16);
  return static_cast<const float*>(table)[idx];
}

// One thread per row: ld bfloat16 inputs written as 16-byte groups.
__global__ __launch_bounds__(kThreads) void tube_points_kernel(TubePointsArgs A) {
  if (A.done && *A.done) return;
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= A.Qc * A.N) return;
  const int64_t q = A.q0 + r / A.N;
  const int i = (int)(r % A.N);
  __bf16* out = A.X0 + r * A.ld;
  for (int c0 = 0; c0 < A.ld; c0 += 8) {
    typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      float val = 0.f;
      if (c < A.n) {
        const float th = A.theta ? A.theta[(int64_t)c * A.Q + q] : 0.f;
        const float y = A.x[(int64_t)c * A.Q + q] + th + A.sigma * table_z(A.table, A.bf16, (int64_t)c * A.tstride + i);
        val = (y - A.mean[c]) / A.stdv[c];
      } else if (c == A.n) {
        val = (A.t_prev - A.mean[c]) / A.stdv[c];
      }
      v[e] = (__bf16)val;
    }
    *reinterpret_cast<bf16x8*>(out + c0) = v;
  }
}

template <int NM>
__global__ __launch_bounds__(kThreads) void tube_lse_kernel(TubeLseArgs A) {
  if (A.done && *A.done) return;
  const int64_t qi = blockIdx.x;
  const int64_t q = A.q0 + qi;
  const int tid = threadIdx.x;
  float th[NM];
  float thn2 = 0.f;
#pragma unroll
  for (int d = 0; d < NM; ++d) {
    th[d] = (A.theta && d < A.n) ? A.theta[(int64_t)d * A.Q + q] : 0.f;
    thn2 = fmaf(th[d], th[d], thn2);
  }
  const float inv_s = 1.0f / A.sigma;
  const float cl = A.c[q] * kLog2e;
  const float a0 = -0.5f * thn2 * inv_s * inv_s * kLog2e;
  const float ts = inv_s * kLog2e;
  const float om = *A.omean, os = *A.ostd;
  float m = -INFINITY, S = 0.f, S2 = 0.f, G[NM];
#pragma unroll
  for (int d = 0; d < NM; ++d) G[d] = 0.f;
  for (int i = tid; i < A.N; i += kThreads) {
    const float ell = fmaf(A.Y[(qi * A.N + i) * A.ldy], os, om);
    float z[NM], zt = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      z[d] = d < A.n ? table_z(A.table, A.bf16, (int64_t)d * A.tstride + i) : 0.f;
      zt = fmaf(z[d], th[d], zt);
    }
    const float a = fmaf(-cl, ell, fmaf(-ts, zt, a0));
    if (a > m) {
      const float f = __builtin_amdgcn_exp2f(m - a);
      S *= f;
      S2 *= f * f;
#pragma unroll
      for (int d = 0; d < NM; ++d) G[d] *= f;
      m = a;
    }
    const float w = __builtin_amdgcn_exp2f(a - m);
    S += w;
    S2 = fmaf(w, w, S2);
#pragma unroll
    for (int d = 0; d < NM; ++d) G[d] = fmaf(w, z[d], G[d]);
  }
  // block maximum, then float64 sums rescaled to it
  __shared__ float smax[kThreads / 64];
  __shared__ double sred[kThreads / 64];
  const int lane = tid & 63, wv = tid >> 6;
  float mx = m;
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) smax[wv] = mx;
  __syncthreads();
  float M = smax[0];
  for (int w = 1; w < kThreads / 64; ++w) M = fmaxf(M, smax[w]);
  const double f = (m == -INFINITY) ? 0.0 : exp2((double)m - (double)M);
  auto block_sum = [&](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) sred[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += sred[w];
    return t;
  };
  const double St = block_sum((double)S * f);
  const double S2t = block_sum((double)S2 * f * f);
  if (tid == 0) {
    A.part.m[q] = M;
    A.part.S[q] = St;
    A.part.S2[q] = S2t;
  }
#pragma unroll
  for (int d = 0; d < NM; ++d) {
    if (d < A.n) {
      const double g = block_sum((double)G[d] * f);
      if (tid == 0) A.part.G[(int64_t)d * A.Q + q] = (float)g;
    }
  }
}

template <int NM>
void lse_launch(const TubeLseArgs& a, hipStream_t s) {
  tube_lse_kernel<NM><<<(unsigned)a.Qc, kThreads, 0, s>>>(a);
}

}  // namespace

hipError_t launch_tube_points(const TubePointsArgs& a, hipStream_t s) {
  const int64_t rows = a.Qc * a.N;
  if (rows <= 0) return hipSuccess;
  tube_points_kernel<<<(unsigned)((rows + kThreads - 1) / kThreads), kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_tube_lse(const TubeLseArgs& a, hipStream_t s) {
  if (a.Qc <= 0) return hipSuccess;
  switch (n_bucket(a.n)) {
    case 4: lse_launch<4>(a, s); break;
    case 8: lse_launch<8>(a, s); break;
    case 16: lse_launch<16>(a, s); break;
    case 32: lse_launch<32>(a, s); break;
    default: lse_launch<48>(a, s); break;
  }
  return hipGetLastError();
}

}  // namespace hjg
