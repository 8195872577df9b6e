// Pair loop with the two dense contractions on the matrix cores (gfx950).
//
// Under common random numbers every query of a tile meets the same samples,
// so per 32 x 32 tile of (samples, queries) the two sums over dimensions are
// small GEMMs on bfloat16 operands with float32 accumulation:
//   T  = Z  Theta^T     T[i][q]  = <z_i, theta_q> log2(e)/sigma   (tilt term)
//   G^T += Z^T W^T      G[d][q]  = sum_i w_qi z_i[d]               (gradient sum)
// with v_mfma_f32_32x32x16_bf16.  The draws are bfloat16 already (exact);
// theta and the weights are split into hi + lo bfloat16 parts so the products
// keep about 16 significant bits.  Everything that is not a contraction --
// y = x + theta + sigma z, the datum l(y), the log-weight, the running
// maximum and exp2 -- stays on the vector ALUs in float32.
//
// Lane layout (verified against the hardware): a wave owns 32 queries; lane l
// serves query l % 32 and half h = l / 32 of every 32-sample group.  The
// accumulator of T gives lane l the tilt term of its own query at samples
// 8(v/4) + 4h + v%4 (v = 0..15), and choosing the K index of the second
// product to run over exactly those samples makes lane l's G accumulators
// belong to its own query too, so the online max-rescale stays lane-local
// (the two halves of a query agree on the maximum through one cross-half
// exchange per group).
#pragma once

#include <type_traits>

#include "kernels.h"

namespace hjg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kMWaves = 4;              // waves per block
constexpr int kMQ = 32 * kMWaves;       // queries per block
constexpr int kMS = 128;                // samples per LDS round

// Number of float32 datum coordinates kept per sample (compile-time bound).
// MP is the exact number of disc pairs for MIN_PAIR_DISKS (n = 3 MP) and is
// unused otherwise; a compile-time count keeps the datum loop free of branches.
template <int DATUM, int NM, int MP>
constexpr int mfma_ndat() {
  return (DATUM == HJG_L_MIN_PAIR_DISKS || DATUM == HJG_L_CAPTURE) ? 2 * MP : (DATUM == HJG_L_LINEAR ? 0 : NM);
}
template <int DATUM, int NM, int MP>
constexpr int mfma_ps() {   // row stride of the float32 table: multiple of 4, +4 against bank conflicts
  return ((mfma_ndat<DATUM, NM, MP>() + 3) / 4) * 4 + 4;
}

template <int DATUM, int NM, int MP>
struct alignas(16) MfmaLds {
  __bf16 sm[kMS][NM + 8];                     // sample-major (A operand of T)
  __bf16 dm[NM][kMS + 8];                     // dimension-major (A operand of G^T)
  float zp[kMS][mfma_ps<DATUM, NM, MP>()];    // datum coordinates, float32
};

// Coordinate slot of dimension d in the float32 datum table, or -1.
template <int DATUM>
__device__ __forceinline__ int datum_slot(const DatumP& dp, int d) {
  if constexpr (DATUM == HJG_L_MIN_PAIR_DISKS || DATUM == HJG_L_CAPTURE) return (d % 3 < 2) ? 2 * (d / 3) + d % 3 : -1;
  else if constexpr (DATUM == HJG_L_BALL) return d < dp.k ? d : -1;
  else if constexpr (DATUM == HJG_L_HALF_SQNORM) return d;
  else return -1;
}

// l(y) for one sample; ud holds x + theta at the datum coordinates and sd the
// per-coordinate sigma (0 where a coordinate does not enter l).
template <int DATUM, int NM, int MP>
__device__ __forceinline__ float mfma_ell(const float* ud, const float* sd, float sg, const DatumP& dp,
                                          const float* zr) {
  if constexpr (DATUM == HJG_L_MIN_PAIR_DISKS) {
    float best = INFINITY;
#pragma unroll
    for (int k = 0; k < MP; ++k) {
      const float y0 = fmaf(sg, zr[2 * k], ud[2 * k]);
      const float y1 = fmaf(sg, zr[2 * k + 1], ud[2 * k + 1]);
      best = fminf(best, fmaf(y0, y0, y1 * y1));
    }
    return __builtin_amdgcn_sqrtf(best) - dp.r;
  } else if constexpr (DATUM == HJG_L_CAPTURE) {
    constexpr int E = MP - 1;                       // the evader is the last agent
    const float ye0 = fmaf(sg, zr[2 * E], ud[2 * E]);
    const float ye1 = fmaf(sg, zr[2 * E + 1], ud[2 * E + 1]);
    float best = INFINITY;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const float y0 = fmaf(sg, zr[2 * k], ud[2 * k]) - ye0;
      const float y1 = fmaf(sg, zr[2 * k + 1], ud[2 * k + 1]) - ye1;
      best = fminf(best, fmaf(y0, y0, y1 * y1));
    }
    return __builtin_amdgcn_sqrtf(best) - dp.r;
  } else if constexpr (DATUM == HJG_L_BALL) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      const float y = fmaf(sd[d], zr[d], ud[d]);
      s = fmaf(y, y, s);
    }
    return __builtin_amdgcn_sqrtf(s) - dp.r;
  } else if constexpr (DATUM == HJG_L_HALF_SQNORM) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      const float y = fmaf(sg, zr[d], ud[d]);
      s = fmaf(y, y, s);
    }
    return 0.5f * s;
  } else {
    return 0.f;   // LINEAR: folded into the contraction
  }
}

template <int DATUM, int NM, int MP>
__device__ __forceinline__ void sweep_mfma_block(const SweepArgs& A, int64_t qblock, int split) {
  constexpr int KS = NM / 16;              // K steps of the tilt product
  constexpr int GT = (NM + 31) / 32;       // 32-dimension tiles of G^T
  constexpr int ND = mfma_ndat<DATUM, NM, MP>();
  constexpr int NDR = ND > 0 ? ND : 1;
  __shared__ MfmaLds<DATUM, NM, MP> L;
  static_assert(sizeof(MfmaLds<DATUM, NM, MP>) <= 64 * 1024, "LDS tile too large");

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ql = lane & 31, h = lane >> 5;
  const int64_t q = qblock * kMQ + wave * 32 + ql;
  const bool active = q < A.Q;
  const int64_t qs = active ? q : A.Q - 1;
  const int i_begin = split * A.ns;
  const int i_end = min(A.N, i_begin + A.ns);
  const bool use_t = (A.theta != nullptr) || DATUM == HJG_L_LINEAR;

  // ---- per-query constants
  const float sg = A.sigma, inv_s = 1.0f / A.sigma;
  float cl = A.c[qs] * kLog2e;
  float a0 = 0.f;
  float ud[NDR], sd[DATUM == HJG_L_BALL ? NM : 1];
#pragma unroll
  for (int s = 0; s < NDR; ++s) ud[s] = 0.f;
  if constexpr (DATUM == HJG_L_BALL) {
#pragma unroll
    for (int d = 0; d < NM; ++d) sd[d] = d < A.dp.k ? A.sigma : 0.f;
  }
  bf16x8_t th_hi[KS], th_lo[KS];
  {
    float thn2 = 0.f, l0 = (DATUM == HJG_L_LINEAR) ? A.dp.r : 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      if (d < A.n) {
        const float xd = A.x[(int64_t)d * A.Q + qs];
        const float th = A.theta ? A.theta[(int64_t)d * A.Q + qs] : 0.f;
        thn2 += th * th;
        if constexpr (ND > 0) {
          const int s = datum_slot<DATUM>(A.dp, d);
#pragma unroll
          for (int k = 0; k < NDR; ++k) if (k == s) ud[k] = xd + th;
        }
        if constexpr (DATUM == HJG_L_LINEAR) l0 += A.dp.aux[d] * (xd + th);
      }
    }
    a0 = -0.5f * thn2 * inv_s * inv_s * kLog2e;
    if constexpr (DATUM == HJG_L_LINEAR) { a0 -= cl * l0; }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int d = 16 * ks + 8 * h + i;
        float tl = 0.f;
        if (d < A.n) {
          const float th = A.theta ? A.theta[(int64_t)d * A.Q + qs] : 0.f;
          tl = th * inv_s * kLog2e;
          if constexpr (DATUM == HJG_L_LINEAR) tl += cl * sg * A.dp.aux[d];
        }
        const __bf16 hi = (__bf16)tl;
        th_hi[ks][i] = hi;
        th_lo[ks][i] = (__bf16)(tl - (float)hi);
      }
    }
    if constexpr (DATUM == HJG_L_LINEAR) cl = 0.f;
  }

  // ---- zero the LDS once: padding dimensions stay zero
  {
    uint32_t* p = reinterpret_cast<uint32_t*>(&L);
    for (int e = tid; e < (int)(sizeof(L) / 4); e += 256) p[e] = 0u;
  }
  __syncthreads();

  float m = -INFINITY, Sb = 0.f, S2b = 0.f;
  double S = 0.0, S2 = 0.0;
  f32x16_t G[GT];
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) G[t][v] = 0.f;

  const __bf16* tab = static_cast<const __bf16*>(A.table);
  for (int i0 = i_begin; i0 < i_end; i0 += kMS) {
    // ---- stage kMS samples x n dimensions in three layouts
    for (int it = tid; it < A.n * (kMS / 8); it += 256) {
      const int d = it / (kMS / 8), c = it % (kMS / 8);
      const int i = i0 + 8 * c;
      bf16x8_t val;
      if (i + 8 <= i_end) {
        val = *reinterpret_cast<const bf16x8_t*>(tab + (int64_t)d * A.tstride + i);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) val[e] = (i + e < i_end) ? tab[(int64_t)d * A.tstride + i + e] : (__bf16)0.f;
      }
      *reinterpret_cast<bf16x8_t*>(&L.dm[d][8 * c]) = val;
#pragma unroll
      for (int e = 0; e < 8; ++e) L.sm[8 * c + e][d] = val[e];
      if constexpr (ND > 0) {
        const int s = datum_slot<DATUM>(A.dp, d);
        if (s >= 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) L.zp[8 * c + e][s] = (float)val[e];
        }
      }
    }
    __syncthreads();

    const int cnt = min(kMS, i_end - i0);
    // full rounds need no per-sample mask; only the ragged last round does
    auto group = [&](int g0, auto masked) {
      // ---- tilt contraction T = Z Theta^T for this 32-sample group
      f32x16_t tz;
#pragma unroll
      for (int v = 0; v < 16; ++v) tz[v] = 0.f;
      if (use_t) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const bf16x8_t za = *reinterpret_cast<const bf16x8_t*>(&L.sm[g0 + ql][16 * ks + 8 * h]);
          tz = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, th_hi[ks], tz, 0, 0, 0);
          tz = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, th_lo[ks], tz, 0, 0, 0);
        }
      }
      // ---- datum and log-weights of the lane's 16 pairs
      float a[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int j = g0 + 8 * (v / 4) + 4 * h + (v % 4);
        const float ell = mfma_ell<DATUM, NM, MP>(ud, sd, sg, A.dp, &L.zp[j][0]);
        const float av = fmaf(-cl, ell, a0 - tz[v]);
        if constexpr (decltype(masked)::value) a[v] = (j < cnt) ? av : -INFINITY;
        else a[v] = av;
      }
      float mb = a[0];
#pragma unroll
      for (int v = 1; v < 16; ++v) mb = fmaxf(mb, a[v]);
      mb = fmaxf(mb, __shfl_xor(mb, 32, 64));     // both halves of the query agree
      if (mb > m) {
        const float sc = __builtin_amdgcn_exp2f(m - mb);
        Sb *= sc;
        S2b *= sc * sc;
        S *= (double)sc;
        S2 *= (double)sc * (double)sc;
#pragma unroll
        for (int t = 0; t < GT; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) G[t][v] *= sc;
        m = mb;
      }
      // ---- weights; gradient contraction G^T += Z^T W^T (hi + lo parts)
#pragma unroll
      for (int kst = 0; kst < 2; ++kst) {
        bf16x8_t whi, wlo;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float w = __builtin_amdgcn_exp2f(a[8 * kst + i] - m);
          Sb += w;
          S2b = fmaf(w, w, S2b);
          const __bf16 hb = (__bf16)w;
          whi[i] = hb;
          wlo[i] = (__bf16)(w - (float)hb);
        }
#pragma unroll
        for (int t = 0; t < GT; ++t) {
          const int dim = 32 * t + ql;
          bf16x8_t za;
          if (dim < NM) {
            const bf16x4_t lo4 = *reinterpret_cast<const bf16x4_t*>(&L.dm[dim][g0 + 16 * kst + 4 * h]);
            const bf16x4_t hi4 = *reinterpret_cast<const bf16x4_t*>(&L.dm[dim][g0 + 16 * kst + 8 + 4 * h]);
#pragma unroll
            for (int e = 0; e < 4; ++e) { za[e] = lo4[e]; za[4 + e] = hi4[e]; }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) za[e] = (__bf16)0.f;
          }
          G[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, whi, G[t], 0, 0, 0);
          G[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, wlo, G[t], 0, 0, 0);
        }
      }
    };
    if (cnt == kMS) {
      for (int g0 = 0; g0 < kMS; g0 += 32) group(g0, std::false_type{});
    } else {
      for (int g0 = 0; g0 < cnt; g0 += 32) group(g0, std::true_type{});
    }
    S += (double)Sb;
    S2 += (double)S2b;
    Sb = S2b = 0.f;
    __syncthreads();
  }

  // ---- combine the two halves of each query and write the split partials
  S += __shfl_xor(S, 32, 64);
  S2 += __shfl_xor(S2, 32, 64);
  if (active) {
    const int64_t sq = (int64_t)split * A.Q + q;
    if (h == 0) {
      A.part.m[sq] = m;
      A.part.S[sq] = S;
      A.part.S2[sq] = S2;
    }
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int dim = 32 * t + 8 * (v / 4) + 4 * h + (v % 4);
        if (dim < A.n) A.part.G[((int64_t)split * A.n + dim) * A.Q + q] = G[t][v];
      }
  }
}

template <int DATUM, int NM, int MP>
__global__ __launch_bounds__(256) void sweep_mfma_kernel(SweepArgs A) {
  if (A.done && *A.done) return;
  sweep_mfma_block<DATUM, NM, MP>(A, blockIdx.x, blockIdx.y);
}

template <int DATUM, int NM, int MP>
__global__ __launch_bounds__(256) void sweep_mfma_batched_kernel(const SweepArgs* probs, const int4* items, int count,
                                                                 int* counter) {
  __shared__ int slot;
  for (int b = counter ? next_item(counter, &slot) : (int)blockIdx.x; b < count;
       b = counter ? next_item(counter, &slot) : count) {
    const int4 it = work_item(items, b);
    const SweepArgs& A = problem_args(probs, it.x);
    if (A.done && *A.done) continue;
    sweep_mfma_block<DATUM, NM, MP>(A, it.y, it.z);
  }
}

}  // namespace hjg
