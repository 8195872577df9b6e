// Device helpers for the HJ-Gauss sweep on gfx950: Philox4x32-10 draws,
// Box-Muller, bfloat16 rounding, terminal data l and Hamiltonians H.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hjg.h"

namespace hjg {

constexpr float kLog2e = 1.4426950408889634f;
constexpr double kLn2 = 0.6931471805599453;
constexpr int kMaxN = 48;
constexpr int kMaxKnn = 8;

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: two 32x32->64 multiplies per round, key advanced by
// the Weyl constants between rounds, ten rounds.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Two normals from a radius word and an angle word:
// u_a = ((wa >> 8) + 1) 2^-24 in (0, 1], u_b = (wb >> 8) 2^-24 in [0, 1),
// r = sqrt(-2 ln u_a), (r cos 2 pi u_b, r sin 2 pi u_b).  Both uniforms are
// exact in float32; the angle goes through sincospi so no range reduction of
// 2 pi u_b is needed.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float ua = (float)((wa >> 8) + 1u) * 5.9604644775390625e-08f;
  const float ub = (float)(wb >> 8) * 5.9604644775390625e-08f;
  const float r = sqrtf(-2.0f * logf(ua));
  float s, c;
  sincospif(2.0f * ub, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// Normals of samples 4g .. 4g+3 in dimension d.
__device__ __forceinline__ void normals4(uint32_t g, uint32_t d, uint32_t stream, uint32_t tag,
                                         uint32_t k0, uint32_t k1, float z[4]) {
  const U4 w = philox4x32_10(U4{g, d, stream, tag}, k0, k1);
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float round_bf16(float f) { return bf16_to_f32(f32_to_bf16_rne(f)); }

// ------------------------------------------------------------------ parameters
// Problem parameters as the kernels see them (float32, resolved on the host).
struct DatumP {
  int kind;       // enum hjg_datum
  int n;          // state dimension
  int k;          // BALL: leading dims; KNN: neighbours
  int m;          // MIN_PAIR_DISKS: pairs; CAPTURE: agents (n / 3)
  float r;        // radius (BALL, MIN_PAIR_DISKS, KNN) or offset b (LINEAR)
  const float* aux;  // LINEAR: a[n]; KNN: [K][3][Q]
};

struct HamP {
  int kind;       // enum hjg_ham
  int n;
  float p[6];
  float inv_delta;      // 1 / delta
  float two_over_delta; // 2 / delta
  float eta, c_min, c_max;
  int tube;             // use min{0, H}
};

// l(x) and D l(x) at one state held in registers (x[d] for d < n).  Same rules
// at kinks as everywhere in the library: radius 0 gives gradient 0; ties in a
// minimum go to the lowest index.
template <int NM>
__device__ inline float datum_and_grad(const DatumP& dp, const float* x, float* g, int64_t q, int64_t Q) {
#pragma unroll
  for (int d = 0; d < NM; ++d) g[d] = 0.f;
  switch (dp.kind) {
    case HJG_L_HALF_SQNORM: {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < NM; ++d) if (d < dp.n) { s += x[d] * x[d]; g[d] = x[d]; }
      return 0.5f * s;
    }
    case HJG_L_BALL: {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < NM; ++d) if (d < dp.k) s += x[d] * x[d];
      const float rho = sqrtf(s);
      if (rho > 0.f) {
#pragma unroll
        for (int d = 0; d < NM; ++d) if (d < dp.k) g[d] = x[d] / rho;
      }
      return rho - dp.r;
    }
    case HJG_L_MIN_PAIR_DISKS: {
      float best = INFINITY;
      int jb = 0;
#pragma unroll
      for (int j = 0; j < NM / 3; ++j) {
        if (j < dp.m) {
          const float r2 = x[3 * j] * x[3 * j] + x[3 * j + 1] * x[3 * j + 1];
          if (r2 < best) { best = r2; jb = j; }
        }
      }
      const float rho = sqrtf(best);
      if (rho > 0.f) {
#pragma unroll
        for (int j = 0; j < NM / 3; ++j) if (j == jb) { g[3 * j] = x[3 * j] / rho; g[3 * j + 1] = x[3 * j + 1] / rho; }
      }
      return rho - dp.r;
    }
    case HJG_L_KNN_BALLS: {
      float best = INFINITY, b0 = 0.f, b1 = 0.f, b2 = 0.f;
      for (int j = 0; j < dp.k; ++j) {
        const float e0 = x[0] - dp.aux[(int64_t)(3 * j + 0) * Q + q];
        const float e1 = x[1] - dp.aux[(int64_t)(3 * j + 1) * Q + q];
        const float e2 = x[2] - dp.aux[(int64_t)(3 * j + 2) * Q + q];
        const float r2 = e0 * e0 + e1 * e1 + e2 * e2;
        if (r2 < best) { best = r2; b0 = e0; b1 = e1; b2 = e2; }
      }
      const float rho = sqrtf(best);
      if (rho > 0.f) { g[0] = b0 / rho; g[1] = b1 / rho; g[2] = b2 / rho; }
      return rho - dp.r;
    }
    case HJG_L_DISC_UNION: {
      float best = INFINITY, b0 = 0.f, b1 = 0.f;
      for (int j = 0; j < dp.k; ++j) {
        const float e0 = x[0] - dp.aux[2 * j], e1 = x[1] - dp.aux[2 * j + 1];
        const float r2 = e0 * e0 + e1 * e1;
        if (r2 < best) { best = r2; b0 = e0; b1 = e1; }
      }
      const float rho = sqrtf(best);
      if (rho > 0.f) { g[0] = b0 / rho; g[1] = b1 / rho; }
      return rho - dp.r;
    }
    case HJG_L_CAPTURE: {
      const int e = dp.m - 1;                        // the evader is the last agent
      float ex = 0.f, ey = 0.f;
#pragma unroll
      for (int j = 0; j < NM / 3; ++j)
        if (j == e) { ex = x[3 * j]; ey = x[3 * j + 1]; }
      float best = INFINITY, bx = 0.f, by = 0.f;
      int jb = 0;
#pragma unroll
      for (int j = 0; j < NM / 3; ++j) {
        if (j < e) {
          const float dx = x[3 * j] - ex, dy = x[3 * j + 1] - ey;
          const float r2 = dx * dx + dy * dy;
          if (r2 < best) { best = r2; jb = j; bx = dx; by = dy; }
        }
      }
      const float rho = sqrtf(best);
      if (rho > 0.f) {
#pragma unroll
        for (int j = 0; j < NM / 3; ++j) {
          if (j == jb) { g[3 * j] = bx / rho; g[3 * j + 1] = by / rho; }
          if (j == e) { g[3 * j] = -bx / rho; g[3 * j + 1] = -by / rho; }
        }
      }
      return rho - dp.r;
    }
    case HJG_L_LINEAR:
    default: {
      float s = dp.r;
#pragma unroll
      for (int d = 0; d < NM; ++d) if (d < dp.n) { s += dp.aux[d] * x[d]; g[d] = dp.aux[d]; }
      return s;
    }
  }
}

// H(x, p) for one state.
template <int NM>
__device__ inline float hamiltonian(const HamP& hp, const float* x, const float* p) {
  switch (hp.kind) {
    case HJG_H_QUADRATIC: {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < NM; ++d) if (d < hp.n) s += p[d] * p[d];
      return 0.5f * s;
    }
    case HJG_H_DUBINS_PAIRS: {
      const float sg = hp.p[0], ve = hp.p[1], vp = hp.p[2], w = hp.p[3];
      float H = 0.f;
#pragma unroll
      for (int j = 0; j < NM / 3; ++j) {
        if (3 * j < hp.n) {
          const float x1 = x[3 * j], x2 = x[3 * j + 1], x3 = x[3 * j + 2];
          const float p1 = p[3 * j], p2 = p[3 * j + 1], p3 = p[3 * j + 2];
          float s3, c3;
          sincosf(x3, &s3, &c3);
          H += p1 * (vp * c3 - ve) + sg * p2 * vp * s3 + w * fabsf(p1 * x2 - p2 * x1 - p3) - w * fabsf(p3);
        }
      }
      return H;
    }
    case HJG_H_PURSUIT_EVASION: {
      const float ae = hp.p[0], ap = hp.p[1], um = hp.p[2];
      const int e = hp.n / 3 - 1;
      float H = 0.f;
#pragma unroll
      for (int j = 0; j < NM / 3; ++j) {
        if (3 * j < hp.n) {
          float s3, c3;
          sincosf(x[3 * j + 2], &s3, &c3);
          const bool ev = j == e;
          H += (ev ? ae : ap) * (p[3 * j] * c3 + p[3 * j + 1] * s3) + (ev ? um : -um) * fabsf(p[3 * j + 2]);
        }
      }
      return H;
    }
    case HJG_H_DOUBLE_INTEGRATOR: {
      // n = 2k: positions x[0..k), velocities x[k..2k); the control term is
      // +u_max |p_vel| (maximising control) or -u_max |p_vel| (ham_p[1] < 0)
      const float um = hp.p[1] < 0.f ? -hp.p[0] : hp.p[0];
      if (hp.n == 2) return p[0] * x[1] + um * fabsf(p[1]);
      if constexpr (NM >= 4) {
        if (hp.n == 4) return p[0] * x[2] + p[1] * x[3] + um * sqrtf(p[2] * p[2] + p[3] * p[3]);
      }
      if constexpr (NM >= 6) {
        const float pv = sqrtf(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
        return p[0] * x[3] + p[1] * x[4] + p[2] * x[5] + um * pv;
      }
      return 0.f;
    }
    case HJG_H_MURMURATION: {
      const float ve = hp.p[0], vp = hp.p[1], we = hp.p[2], wp = hp.p[3], glo = hp.p[4], ghi = hp.p[5];
      float s4, c4;
      sincosf(x[3], &s4, &c4);
      return p[0] * (ve - vp * c4) - p[1] * vp * s4 - wp * fabsf(p[3]) + we * fabsf(p[1] * x[0] - p[0] * x[1] + p[3]) +
             (glo - ghi) * fabsf(p[2]);
    }
    case HJG_H_ROCKETS: {
      // relative rockets: x' = a cos th + u_e x, z' = a sin th + a + u_p x - g,
      // th' = u_p - u_e; H = -max_{u_e} min_{u_p} <p, f>
      const float a = hp.p[0], g = hp.p[1], um = hp.p[2];
      float s3, c3;
      sincosf(x[2], &s3, &c3);
      return -(a * p[0] * c3 + p[1] * (a + a * s3 - g) + um * fabsf(p[0] * x[0] - p[2]) -
               um * fabsf(p[1] * x[0] + p[2]));
    }
    case HJG_H_ZERO:
    default:
      return 0.f;
  }
}

// Frozen coefficient: c = (2/delta) H / (|p|^2 + eta), |c| clipped to
// [c_min, c_max], sign kept, sign(0) = +1; exactly 1/delta for H = |p|^2/2.
// The tube equation uses min{0, H} in place of H.
template <int NM>
__device__ inline float coefficient(const HamP& hp, const float* x, const float* p) {
  if (hp.kind == HJG_H_QUADRATIC) return hp.inv_delta;
  float pp = 0.f;
#pragma unroll
  for (int d = 0; d < NM; ++d) if (d < hp.n) pp += p[d] * p[d];
  float H = hamiltonian<NM>(hp, x, p);
  if (hp.tube) H = fminf(H, 0.f);
  const float raw = hp.two_over_delta * H / (pp + hp.eta);
  const float mag = fminf(fmaxf(fabsf(raw), hp.c_min), hp.c_max);
  return raw < 0.f ? -mag : mag;
}

}  // namespace hjg
