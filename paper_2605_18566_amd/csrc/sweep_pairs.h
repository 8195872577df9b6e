// Pair loop for stacked disc pairs with the contractions on the matrix cores,
// one query per lane (gfx950).
//
// The datum of m stacked pairs needs 2m float32 coordinates of every sample
// (the planar offsets of each pair); everything else a pair needs is one
// value per query.  A wave owns 64 queries, one per lane, and walks the
// samples of a 32-sample group together, so each sample's coordinates are the
// same for every lane: they come into scalar registers from a float32
// sample-major copy made with the draw table, and each offset
// y = sigma z + (x + theta) is one full-rate FMA with a scalar operand (no
// per-lane LDS traffic, no cross-lane broadcast instruction).  The next
// sample's coordinates are requested right after the wait for the current
// ones, so the scalar-cache latency hides behind one sample of arithmetic
// (scheduling barriers keep the compiler from moving the request).
//
// The two contractions stay on v_mfma_f32_32x32x16_bf16 (bfloat16 operands,
// float32 accumulation; theta and the weights split into hi + lo parts):
//   T  = Z Theta^T  for the wave's two 32-query tiles (queries 0..31, 32..63)
//   G^T += Z^T W^T  for the same two tiles.
// An MFMA result gives lane l query l % 32 at samples 8(v/4) + 4h + v%4
// (h = l / 32): each query's 32 samples are split over lanes l and l + 32.
// One v_permlane32_swap per register exchanges tile B's h = 0 values with
// tile A's h = 1 values, after which lane l holds all 32 samples of query l
// (lanes 0..31 tile A, lanes 32..63 tile B); the same swap on the packed
// weights builds the B operands of both tiles of the gradient product.
#pragma once

#include <cstddef>

#include "sweep_mfma.h"

namespace hjg {

constexpr int kPWaves = 8;              // waves per block
constexpr int kPThreads = 64 * kPWaves;
constexpr int kPQ = 64 * kPWaves;       // queries per block
static_assert(kPQ == kQueriesPerBlockPairs, "host and kernel disagree on queries per block");

template <int NM>
struct alignas(16) PairsLds {
  __bf16 sm[kMS][NM + 8];   // sample-major (A operand of T)
  __bf16 dm[NM][kMS + 8];   // dimension-major (A operand of G^T)
  // B operands of T per wave: [tile][k step][hi, lo][lane]
  bf16x8_t th[kPWaves][2][NM / 16][2][64];
};

__device__ __forceinline__ uint32_t swap_hi_lo(uint32_t& x, uint32_t y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  return r[1];
}

__device__ __forceinline__ void swap_halves(float& a, float& b) {
  uint32_t x = __float_as_uint(a);
  const uint32_t y = swap_hi_lo(x, __float_as_uint(b));
  a = __uint_as_float(x);
  b = __uint_as_float(y);
}

__device__ __forceinline__ void swap_halves(bf16x8_t& a, bf16x8_t& b) {
  typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4_t;
  u32x4_t x = __builtin_bit_cast(u32x4_t, a), y = __builtin_bit_cast(u32x4_t, b);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t xi = x[i];
    y[i] = swap_hi_lo(xi, y[i]);
    x[i] = xi;
  }
  a = __builtin_bit_cast(bf16x8_t, x);
  b = __builtin_bit_cast(bf16x8_t, y);
}

typedef const float __attribute__((address_space(4)))* const_f32_p;

// Minimum of v[0..N) as a tree of three-way minima (depth log3 N instead of a
// chain of N/2 dependent min3).
template <int N>
__device__ __forceinline__ float min_tree(const float* v) {
  if constexpr (N == 1) {
    return v[0];
  } else if constexpr (N == 2) {
    return fminf(v[0], v[1]);
  } else {
    constexpr int G = (N + 2) / 3;
    float w[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int b = 3 * g;
      w[g] = b + 2 < N ? fminf(fminf(v[b], v[b + 1]), v[b + 2]) : (b + 1 < N ? fminf(v[b], v[b + 1]) : v[b]);
    }
    return min_tree<G>(w);
  }
}

template <int NM, int MP>
__device__ __forceinline__ void sweep_pairs_block(const SweepArgs& A, int64_t qblock, int split) {
  constexpr int KS = NM / 16;
  constexpr int GT = (NM + 31) / 32;
  constexpr int NSL = 2 * MP;                 // coordinates per sample
  constexpr int ZS = pair_coord_stride(MP);   // floats per row of the copy
  __shared__ PairsLds<NM> L;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ql = lane & 31, h = lane >> 5;
  const int64_t qw = qblock * kPQ + wave * 64;           // first query of the wave
  const int64_t q = qw + lane;                            // this lane's own query
  const bool active = q < A.Q;
  const int64_t qs = active ? q : A.Q - 1;
  const int64_t qa = min(qw + ql, A.Q - 1);               // tile A query of this lane
  const int64_t qb = min(qw + 32 + ql, A.Q - 1);          // tile B query of this lane
  const int i_begin = split * A.ns;
  const int i_end = min(A.N, i_begin + A.ns);
  const bool use_t = A.theta != nullptr;

  // ---- own query: x + theta at the datum coordinates, c log2(e), constant of a
  const float inv_s = 1.0f / A.sigma;
  // sigma in a vector register: the sample coordinate is the one scalar
  // operand each offset FMA may take
  float sg;
  asm("v_mov_b32 %0, %1" : "=v"(sg) : "s"(A.sigma));
  const float cl = A.c[qs] * kLog2e;
  float us[NSL];
#pragma unroll
  for (int k = 0; k < NSL; ++k) us[k] = 0.f;
  float a0;
  {
    float thn2 = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      if (d < A.n) {
        const float th = use_t ? A.theta[(int64_t)d * A.Q + qs] : 0.f;
        thn2 += th * th;
        if (d % 3 < 2 && d / 3 < MP) us[2 * (d / 3) + d % 3] = A.x[(int64_t)d * A.Q + qs] + th;
      }
    }
    a0 = -0.5f * thn2 * inv_s * inv_s * kLog2e;
  }

  // ---- zero the sample tiles once: padding dimensions stay zero
  {
    uint32_t* p = reinterpret_cast<uint32_t*>(&L);
    for (int e = tid; e < (int)(offsetof(PairsLds<NM>, th) / 4); e += kPThreads) p[e] = 0u;
  }
  // ---- B operands of T for the two tiles, log2(e) theta / sigma as hi + lo,
  // kept in LDS (each wave reads back only what it wrote, after the barrier
  // that ends the first staging round)
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8_t ah, al, bh, bl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int d = 16 * ks + 8 * h + i;
      float ta = 0.f, tb = 0.f;
      if (d < A.n && use_t) {
        ta = A.theta[(int64_t)d * A.Q + qa] * inv_s * kLog2e;
        tb = A.theta[(int64_t)d * A.Q + qb] * inv_s * kLog2e;
      }
      const __bf16 ha = (__bf16)ta, hb = (__bf16)tb;
      ah[i] = ha;
      al[i] = (__bf16)(ta - (float)ha);
      bh[i] = hb;
      bl[i] = (__bf16)(tb - (float)hb);
    }
    L.th[wave][0][ks][0][lane] = ah;
    L.th[wave][0][ks][1][lane] = al;
    L.th[wave][1][ks][0][lane] = bh;
    L.th[wave][1][ks][1][lane] = bl;
  }
  __syncthreads();

  float m = -INFINITY, Sb = 0.f, S2b = 0.f;
  double S = 0.0, S2 = 0.0;
  f32x16_t GA[GT], GB[GT];
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) GA[t][v] = GB[t][v] = 0.f;

  const __bf16* tab = static_cast<const __bf16*>(A.table);
  const const_f32_p zc = (const_f32_p)A.zd;
  for (int i0 = i_begin; i0 < i_end; i0 += kMS) {
    // ---- stage kMS samples x n dimensions in both bf16 layouts
    for (int it = tid; it < A.n * (kMS / 8); it += kPThreads) {
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
    }
    __syncthreads();

    const int cnt = min(kMS, i_end - i0);
    auto group = [&](int g0, auto masked) {
      const const_f32_p zg = zc + (int64_t)(i0 + g0) * ZS;   // the group's first sample row
      // ---- tilt contraction for both tiles, then regroup by own query
      f32x16_t ta, tb;
#pragma unroll
      for (int v = 0; v < 16; ++v) ta[v] = tb[v] = 0.f;
      if (use_t) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const bf16x8_t za = *reinterpret_cast<const bf16x8_t*>(&L.sm[g0 + ql][16 * ks + 8 * h]);
          ta = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, L.th[wave][0][ks][0][lane], ta, 0, 0, 0);
          ta = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, L.th[wave][0][ks][1][lane], ta, 0, 0, 0);
          tb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, L.th[wave][1][ks][0][lane], tb, 0, 0, 0);
          tb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, L.th[wave][1][ks][1][lane], tb, 0, 0, 0);
        }
      }
      float a[32];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float x0 = ta[v], x1 = tb[v];
        swap_halves(x0, x1);
        a[v] = x0;        // sample 8(v/4) + v%4
        a[16 + v] = x1;   // sample 8(v/4) + 4 + v%4
      }
      // ---- datum and log-weights of the lane's 32 pairs.  Sample u's offsets
      // and squared radii are computed in the same scheduling region as the
      // square root and log-weight of sample u - 1, so the dependent tail of
      // one sample overlaps the independent arithmetic of the next.
      auto coords = [&](int u) {
        const int j = g0 + 8 * ((u & 15) / 4) + 4 * (u / 16) + (u & 3);
        if constexpr (decltype(masked)::value) {
          const int64_t row = j < cnt ? i0 + j : i_end - 1;
          return zc + row * ZS;
        } else {
          return zg + (8 * ((u & 15) / 4) + 4 * (u / 16) + (u & 3)) * ZS;
        }
      };
      auto finish = [&](int u, float mn) {
        const float ell = __builtin_amdgcn_sqrtf(mn) - A.dp.r;
        const float av = fmaf(-cl, ell, a0 - a[u]);
        if constexpr (decltype(masked)::value) {
          const int j = g0 + 8 * ((u & 15) / 4) + 4 * (u / 16) + (u & 3);
          a[u] = (j < cnt) ? av : -INFINITY;
        } else {
          a[u] = av;
        }
      };
      float zcur[NSL], znext[NSL];
      {
        const const_f32_p zr = coords(0);
#pragma unroll
        for (int k = 0; k < NSL; ++k) zcur[k] = zr[k];
      }
      float mn_prev = 0.f;
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        // the first use waits for this sample's coordinates; only then is the
        // next sample's request issued (scalar loads return out of order, so
        // any wait covers every request in flight)
        const float y00 = fmaf(sg, zcur[0], us[0]);
        __builtin_amdgcn_sched_barrier(0);
        if (u + 1 < 32) {
          const const_f32_p zr = coords(u + 1);
#pragma unroll
          for (int k = 0; k < NSL; ++k) znext[k] = zr[k];
        }
        __builtin_amdgcn_sched_barrier(0);
        float r2[MP];
        {
          const float y01 = fmaf(sg, zcur[1], us[1]);
          r2[0] = fmaf(y00, y00, y01 * y01);
        }
#pragma unroll
        for (int k = 1; k < MP; ++k) {
          const float y0 = fmaf(sg, zcur[2 * k], us[2 * k]);
          const float y1 = fmaf(sg, zcur[2 * k + 1], us[2 * k + 1]);
          r2[k] = fmaf(y0, y0, y1 * y1);
        }
        if (u > 0) finish(u - 1, mn_prev);
        mn_prev = min_tree<MP>(r2);
        if (u + 1 < 32) {
#pragma unroll
          for (int k = 0; k < NSL; ++k) zcur[k] = znext[k];
        }
      }
      finish(31, mn_prev);
      float mb = a[0];
#pragma unroll
      for (int u = 1; u < 32; ++u) mb = fmaxf(mb, a[u]);
      // rescale to the new maximum; the gradient sums of a lane belong to
      // queries qw + ql (tile A) and qw + 32 + ql (tile B), one of them the
      // partner lane's, so each takes the factor of its own query
      const float m_new = fmaxf(m, mb);
      const float sc = __builtin_amdgcn_exp2f(m - m_new);
      float sca = sc, scb = sc;
      swap_halves(sca, scb);          // sca: factor of query qw + ql, scb: of qw + 32 + ql
      if (m_new > m) {
        Sb *= sc;
        S2b *= sc * sc;
        S *= (double)sc;
        S2 *= (double)sc * (double)sc;
        m = m_new;
      }
      if (sca < 1.f || scb < 1.f) {
#pragma unroll
        for (int t = 0; t < GT; ++t)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            GA[t][v] *= sca;
            GB[t][v] *= scb;
          }
      }
      // ---- weights; gradient contraction for both tiles (K = 16 samples per step)
#pragma unroll
      for (int kst = 0; kst < 2; ++kst) {
        bf16x8_t xh, xl, yh, yl;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float wx = __builtin_amdgcn_exp2f(a[8 * kst + i] - m);
          const float wy = __builtin_amdgcn_exp2f(a[16 + 8 * kst + i] - m);
          Sb += wx + wy;
          S2b = fmaf(wx, wx, fmaf(wy, wy, S2b));
          const __bf16 hx = (__bf16)wx, hy = (__bf16)wy;
          xh[i] = hx;
          xl[i] = (__bf16)(wx - (float)hx);
          yh[i] = hy;
          yl[i] = (__bf16)(wy - (float)hy);
        }
        // x: tile A operand (own query's first samples on h = 0, partner's on h = 1);
        // y: tile B operand
        swap_halves(xh, yh);
        swap_halves(xl, yl);
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
          GA[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, xh, GA[t], 0, 0, 0);
          GA[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, xl, GA[t], 0, 0, 0);
          GB[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, yh, GB[t], 0, 0, 0);
          GB[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, yl, GB[t], 0, 0, 0);
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

  // ---- split partials: own query's sums, both tiles' gradient sums
  const int64_t sbase = (int64_t)split * A.Q;
  if (active) {
    A.part.m[sbase + q] = m;
    A.part.S[sbase + q] = S;
    A.part.S2[sbase + q] = S2;
  }
  // tile A's sums are relative to the maximum of query qw + ql (held by lane
  // ql), tile B's to that of qw + 32 + ql (lane 32 + ql)
  const int64_t qA = qw + ql, qB = qw + 32 + ql;
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int dim = 32 * t + 8 * (v / 4) + 4 * h + (v % 4);
      if (dim < A.n) {
        if (qA < A.Q) A.part.G[((int64_t)split * A.n + dim) * A.Q + qA] = GA[t][v];
        if (qB < A.Q) A.part.G[((int64_t)split * A.n + dim) * A.Q + qB] = GB[t][v];
      }
    }
}

template <int NM, int MP>
__global__ __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(2))) void sweep_pairs_kernel(SweepArgs A) {
  if (A.done && *A.done) return;
  sweep_pairs_block<NM, MP>(A, blockIdx.x, blockIdx.y);
}

template <int NM, int MP>
__global__ __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(2))) void sweep_pairs_batched_kernel(
    const SweepArgs* probs, const int4* items, int count, int* counter) {
  __shared__ int slot;
  for (int b = counter ? next_item(counter, &slot) : (int)blockIdx.x; b < count;
       b = counter ? next_item(counter, &slot) : count) {
    const int4 it = work_item(items, b);
    const SweepArgs& A = problem_args(probs, it.x);
    if (A.done && *A.done) continue;
    sweep_pairs_block<NM, MP>(A, it.y, it.z);
  }
}

}  // namespace hjg
