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
        const float y = fmaf(A.sigma, table_z(A.table, A.bf16, (int64_t)c * A.tstride + i), A.x[(int64_t)c * A.Q + q] + th);
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

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

__device__ __forceinline__ float sigmoid_rcp(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

constexpr int kFR = 128;          // samples per tile: 4 waves x 32
constexpr int kFW = 128;          // hidden width
constexpr int kFK = 32;           // padded input width
constexpr int kHS = kFW + 8;      // LDS row strides (bfloat16), 16-byte aligned rows
constexpr int kXS = kFK + 8;

// One layer for the tile: wave w computes features f0..f0+31 of all 128
// samples as D[f][s] = sum_k W[f][k] H[s][k] (A operand = the wave's weight
// rows in registers, B operand = activation rows from LDS), so that a lane
// holds one sample; bias and SiLU, then bfloat16 rows back to LDS.
// Accumulator lane l: sample 32 st + l % 32, features 8(v/4) + 4(l/32) + v%4.
template <int K, int LD>
__device__ __forceinline__ void fused_layer(const __bf16* Hin, const bf16x8_t* wreg, const float* bias, __bf16* Hout,
                                            int f0, int l32, int h) {
  // accumulators start at the bias of their feature (rows 8(v/4) + 4h + v%4)
  float4 bv[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) bv[g] = *reinterpret_cast<const float4*>(bias + f0 + 8 * g + 4 * h);
  f32x16_t acc[4];
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[st][v] = bv[v / 4][v % 4];
#pragma unroll
  for (int ks = 0; ks < K / 16; ++ks) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(Hin + (32 * st + l32) * LD + 16 * ks + 8 * h);
      acc[st] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wreg[ks], b, acc[st], 0, 0, 0);
    }
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      bf16x4_t o;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float z = acc[st][4 * g + j];
        o[j] = (__bf16)(z * sigmoid_rcp(z));
      }
      *reinterpret_cast<bf16x4_t*>(Hout + (32 * st + l32) * kHS + f0 + 8 * g + 4 * h) = o;
    }
  }
}

template <int D, int NM>
__global__ __launch_bounds__(kThreads, 2) void tube_fused_kernel(TubeFusedArgs A) {
  __shared__ __attribute__((aligned(16))) __bf16 X0[kFR * kXS];
  __shared__ __attribute__((aligned(16))) __bf16 H[2][kFR * kHS];
  __shared__ __attribute__((aligned(16))) float Bs[D][kFW];
  __shared__ float smax[kThreads / 64];
  __shared__ double sred[kThreads / 64];
  if (A.done && *A.done) return;
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l32 = lane & 31, h = lane >> 5;
  const int f0 = 32 * wv;
  for (int e = tid; e < D * kFW; e += kThreads) Bs[e / kFW][e % kFW] = A.b[e / kFW][e % kFW];
  // A operands: the wave's 32 features of each hidden layer, rows 0..31 of the output layer
  bf16x8_t w0[kFK / 16];
#pragma unroll
  for (int ks = 0; ks < kFK / 16; ++ks)
    w0[ks] = *reinterpret_cast<const bf16x8_t*>(A.W[0] + (int64_t)(f0 + l32) * kFK + 16 * ks + 8 * h);
  bf16x8_t wh[D > 1 ? D - 1 : 1][kFW / 16];
#pragma unroll
  for (int l = 1; l < D; ++l)
#pragma unroll
    for (int ks = 0; ks < kFW / 16; ++ks)
      wh[l - 1][ks] = *reinterpret_cast<const bf16x8_t*>(A.W[l] + (int64_t)(f0 + l32) * kFW + 16 * ks + 8 * h);
  const float bo = A.b[D][0];
  const float om = *A.omean, os = *A.ostd;
  // the query: x, theta, constants of the log-weight, the time input
  float xq[NM], th[NM];
  float thn2 = 0.f;
#pragma unroll
  for (int d = 0; d < NM; ++d) {
    xq[d] = d < A.n ? A.x[(int64_t)d * A.Q + q] : 0.f;
    th[d] = (A.theta && d < A.n) ? A.theta[(int64_t)d * A.Q + q] : 0.f;
    thn2 = fmaf(th[d], th[d], thn2);
  }
  const float inv_s = 1.0f / A.sigma;
  const float cl = A.c[q] * kLog2e;
  const float a0 = -0.5f * thn2 * inv_s * inv_s * kLog2e;
  const float ts = inv_s * kLog2e;
  const float tin = (A.t_prev - A.mean[A.n]) / A.stdv[A.n];
  float m = -INFINITY, S = 0.f, S2 = 0.f, G[NM];
#pragma unroll
  for (int d = 0; d < NM; ++d) G[d] = 0.f;
  __syncthreads();
  for (int i0 = 0; i0 < A.N; i0 += kFR) {
    const int s = 32 * wv + l32;       // the lane's sample in the tile (lanes with h = 0 own it)
    const int i = i0 + s;
    const bool valid = i < A.N;
    float z[NM];
    float zt = 0.f;
    if (h == 0) {
#pragma unroll
      for (int d = 0; d < NM; ++d) {
        z[d] = (d < A.n && valid) ? table_z(A.table, A.bf16, (int64_t)d * A.tstride + i) : 0.f;
        zt = fmaf(z[d], th[d], zt);
      }
#pragma unroll
      for (int c0 = 0; c0 < kFK; c0 += 8) {
        bf16x8_t v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = c0 + e;
          float val = 0.f;
          if (c < NM && c < A.n) val = (fmaf(A.sigma, z[c < NM ? c : 0], xq[c < NM ? c : 0] + th[c < NM ? c : 0]) -
                                        A.mean[c]) / A.stdv[c];
          else if (c == A.n) val = tin;
          v[e] = (__bf16)val;
        }
        *reinterpret_cast<bf16x8_t*>(&X0[s * kXS + c0]) = v;
      }
    }
    __syncthreads();
    fused_layer<kFK, kXS>(X0, w0, Bs[0], H[0], f0, l32, h);
    __syncthreads();
#pragma unroll
    for (int l = 1; l < D; ++l) {
      fused_layer<kFW, kHS>(H[(l - 1) & 1], wh[l - 1], Bs[l], H[l & 1], f0, l32, h);
      __syncthreads();
    }
    // value output of the wave's sample tile: feature 0 is accumulator 0 of lanes h = 0
    f32x16_t acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    const __bf16* Hl = H[(D - 1) & 1];
#pragma unroll
    for (int ks = 0; ks < kFW / 16; ++ks) {
      // output-layer rows come from the cache each tile (registers are spent on the hidden layers)
      const bf16x8_t wo = *reinterpret_cast<const bf16x8_t*>(A.W[D] + (int64_t)l32 * kFW + 16 * ks + 8 * h);
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(Hl + (32 * wv + l32) * kHS + 16 * ks + 8 * h);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wo, b, acc, 0, 0, 0);
    }
    if (h == 0 && valid) {
      const float ell = fmaf(acc[0] + bo, os, om);
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
  }
  // block maximum, then float64 sums rescaled to it
  float mx = m;
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) smax[wv] = mx;
  __syncthreads();
  float M = smax[0];
  for (int k = 1; k < kThreads / 64; ++k) M = fmaxf(M, smax[k]);
  const double f = (m == -INFINITY) ? 0.0 : exp2((double)m - (double)M);
  auto block_sum = [&](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) sred[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += sred[k];
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

template <int D>
void fused_launch_d(const TubeFusedArgs& a, hipStream_t s) {
  const unsigned grid = (unsigned)a.Q;
  if (a.n <= 4) tube_fused_kernel<D, 4><<<grid, kThreads, 0, s>>>(a);
  else tube_fused_kernel<D, 8><<<grid, kThreads, 0, s>>>(a);
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

hipError_t launch_tube_fused(const TubeFusedArgs& a, hipStream_t s) {
  if (a.Q <= 0) return hipSuccess;
  if (a.n > kTubeFusedMaxN || a.depth < 1 || a.depth > kTubeFusedMaxDepth) return hipErrorInvalidValue;
  switch (a.depth) {
    case 1: fused_launch_d<1>(a, s); break;
    case 2: fused_launch_d<2>(a, s); break;
    default: fused_launch_d<3>(a, s); break;
  }
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
