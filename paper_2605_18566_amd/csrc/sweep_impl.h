// Pair-loop kernels of one frozen-coefficient sweep.
//
// Work decomposition: one thread per evaluation state (query), 256 queries
// per block, the N samples cut into `splits` contiguous ranges along
// blockIdx.y.  With a common table (CRN) the block stages 128 samples x n
// dimensions of the table in LDS per round and every lane reads the same
// sample at the same time (LDS broadcast, no bank conflicts); with fresh draws
// each lane runs Philox for its own query in registers.
//
// Per pair the lane forms the log2 weight
//   a = log2(e) * (-c l(y) - |theta|^2/(2 sigma^2) - <z, theta>/sigma),
//   y = x + theta + sigma z
// and keeps a running maximum m; per round it accumulates in float32
//   S = sum 2^(a-m), S2 = sum 2^(2(a-m)), G[d] = sum 2^(a-m) z[d]
// and folds S, S2 into float64 at the end of each LDS round (the cross-block
// part of the log-sum-exp merge).
#pragma once

#include <algorithm>

#include "kernels.h"
#include "sweep_mfma.h"
#include "sweep_pairs.h"

namespace hjg {

// Coordinates that never win a minimum: padded disc pairs and neighbours are
// centred this far away, so the datum loops need no branch on the runtime
// pair or neighbour count (1e18^2 stays finite in float32).
constexpr float kFar = 1e18f;

template <int DATUM, int NM>
struct PairConst {
  float u[NM];    // x + theta, the proposal mean (kFar on padded disc pairs)
  float tl[NM];   // log2(e) theta / sigma (LINEAR: also folds in the datum slope)
  float nb[DATUM == HJG_L_KNN_BALLS ? 3 * kMaxKnn : (DATUM == HJG_L_DISC_UNION ? 2 * kMaxKnn : 1)];
                  // x + theta - neighbour (KNN) or - planar centre (DISC_UNION)
  float sd[DATUM == HJG_L_BALL ? NM : 1];                // sigma on the ball's k coordinates, else 0
  float sg;       // sigma
  float cl;       // log2(e) c
  float a0;       // constant part of a
};

template <int DATUM, int NM>
__device__ __forceinline__ void pair_setup(PairConst<DATUM, NM>& P, const SweepArgs& A, int64_t q) {
  const float inv_s = 1.0f / A.sigma;
  const float c = A.c[q];
  P.sg = A.sigma;
  P.cl = c * kLog2e;
  float thn2 = 0.f;
#pragma unroll
  for (int d = 0; d < NM; ++d) {
    float th = 0.f, xd = 0.f;
    if (d < A.n) {
      xd = A.x[(int64_t)d * A.Q + q];
      if (A.theta) th = A.theta[(int64_t)d * A.Q + q];
    }
    P.u[d] = xd + th;
    P.tl[d] = th * inv_s * kLog2e;
    thn2 += th * th;
  }
  P.a0 = -0.5f * thn2 * inv_s * inv_s * kLog2e;
  if constexpr (DATUM == HJG_L_KNN_BALLS) {
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j)
#pragma unroll
      for (int e = 0; e < 3; ++e)
        P.nb[3 * j + e] = (j < A.dp.k) ? P.u[e] - A.dp.aux[(int64_t)(3 * j + e) * A.Q + q] : kFar;
  }
  if constexpr (DATUM == HJG_L_DISC_UNION) {
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j)
#pragma unroll
      for (int e = 0; e < 2; ++e) P.nb[2 * j + e] = (j < A.dp.k) ? P.u[e] - A.dp.aux[2 * j + e] : kFar;
  }
  if constexpr (DATUM == HJG_L_MIN_PAIR_DISKS) {
#pragma unroll
    for (int d = 0; d < NM; ++d)
      if (d >= A.n) P.u[d] = kFar;
  }
  if constexpr (DATUM == HJG_L_BALL) {
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      P.sd[d] = d < A.dp.k ? A.sigma : 0.f;
      if (d >= A.dp.k) P.u[d] = 0.f;
    }
  }
  if constexpr (DATUM == HJG_L_LINEAR) {
    // l(y) = b + <a, u> + sigma <a, z>: the z-part joins the tilt contraction.
    float l0 = A.dp.r;
#pragma unroll
    for (int d = 0; d < NM; ++d)
      if (d < A.n) {
        l0 += A.dp.aux[d] * P.u[d];
        P.tl[d] += P.cl * A.sigma * A.dp.aux[d];
      }
    P.a0 -= P.cl * l0;
    P.cl = 0.f;
  }
}

// log2 weight of one pair; zf(d) returns the sample's coordinate d (0 beyond n).
// MP is the number of disc pairs evaluated (MIN_PAIR_DISKS): the exact count
// or NM/3 with the padded pairs centred at kFar.
template <int DATUM, int NM, int MP, class ZF>
__device__ __forceinline__ float pair_log2w(const PairConst<DATUM, NM>& P, const DatumP& dp, ZF zf) {
  float tz = 0.f;
  float ell = 0.f;
  if constexpr (DATUM == HJG_L_HALF_SQNORM) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      const float z = zf(d);
      const float y = fmaf(P.sg, z, P.u[d]);
      s = fmaf(y, y, s);
      tz = fmaf(z, P.tl[d], tz);
    }
    ell = 0.5f * s;
  } else if constexpr (DATUM == HJG_L_BALL) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      const float z = zf(d);
      const float y = fmaf(P.sd[d], z, P.u[d]);
      s = fmaf(y, y, s);
      tz = fmaf(z, P.tl[d], tz);
    }
    ell = __builtin_amdgcn_sqrtf(s) - dp.r;
  } else if constexpr (DATUM == HJG_L_MIN_PAIR_DISKS) {
    float best = INFINITY;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      const float z0 = zf(3 * j), z1 = zf(3 * j + 1), z2 = zf(3 * j + 2);
      const float y0 = fmaf(P.sg, z0, P.u[3 * j]);
      const float y1 = fmaf(P.sg, z1, P.u[3 * j + 1]);
      best = fminf(best, fmaf(y0, y0, y1 * y1));
      tz = fmaf(z0, P.tl[3 * j], tz);
      tz = fmaf(z1, P.tl[3 * j + 1], tz);
      tz = fmaf(z2, P.tl[3 * j + 2], tz);
    }
    ell = __builtin_amdgcn_sqrtf(best) - dp.r;
  } else if constexpr (DATUM == HJG_L_CAPTURE) {
    // MP agents, the last the evader: min over pursuers of |y_j - y_evader|
    constexpr int E = MP - 1;
    const float ye0 = fmaf(P.sg, zf(3 * E), P.u[3 * E]);
    const float ye1 = fmaf(P.sg, zf(3 * E + 1), P.u[3 * E + 1]);
    float best = INFINITY;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const float y0 = fmaf(P.sg, zf(3 * j), P.u[3 * j]) - ye0;
      const float y1 = fmaf(P.sg, zf(3 * j + 1), P.u[3 * j + 1]) - ye1;
      best = fminf(best, fmaf(y0, y0, y1 * y1));
    }
#pragma unroll
    for (int d = 0; d < 3 * MP; ++d) tz = fmaf(zf(d), P.tl[d], tz);
    ell = __builtin_amdgcn_sqrtf(best) - dp.r;
  } else if constexpr (DATUM == HJG_L_KNN_BALLS) {
    const float z0 = zf(0), z1 = zf(1), z2 = zf(2);
    const float s0 = P.sg * z0, s1 = P.sg * z1, s2 = P.sg * z2;
    float best = INFINITY;
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) {
      const float e0 = P.nb[3 * j] + s0, e1 = P.nb[3 * j + 1] + s1, e2 = P.nb[3 * j + 2] + s2;
      best = fminf(best, fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
    }
#pragma unroll
    for (int d = 0; d < NM; ++d) tz = fmaf(zf(d), P.tl[d], tz);
    ell = __builtin_amdgcn_sqrtf(best) - dp.r;
  } else if constexpr (DATUM == HJG_L_DISC_UNION) {
    const float s0 = P.sg * zf(0), s1 = P.sg * zf(1);
    float best = INFINITY;
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) {
      const float e0 = P.nb[2 * j] + s0, e1 = P.nb[2 * j + 1] + s1;
      best = fminf(best, fmaf(e0, e0, e1 * e1));
    }
#pragma unroll
    for (int d = 0; d < NM; ++d) tz = fmaf(zf(d), P.tl[d], tz);
    ell = __builtin_amdgcn_sqrtf(best) - dp.r;
  } else {  // LINEAR: everything is in the contraction
#pragma unroll
    for (int d = 0; d < NM; ++d) tz = fmaf(zf(d), P.tl[d], tz);
  }
  return fmaf(-P.cl, ell, P.a0 - tz);
}

// Running log-sum-exp state of one lane.
template <int NM>
struct LseAcc {
  float m;
  float Sb, S2b;   // float32 sums of the current LDS round
  double S, S2;    // float64 totals of finished rounds
  float g[NM];
  float zs[NM];    // FRESH control variate: sum z
};

template <int NM>
__device__ __forceinline__ void lse_init(LseAcc<NM>& L) {
  L.m = -INFINITY;
  L.Sb = L.S2b = 0.f;
  L.S = L.S2 = 0.0;
#pragma unroll
  for (int d = 0; d < NM; ++d) L.g[d] = L.zs[d] = 0.f;
}

// Raise the running maximum to mb (if larger) and rescale everything kept so far.
template <int NM>
__device__ __forceinline__ void lse_rebase(LseAcc<NM>& L, float mb) {
  if (mb > L.m) {
    const float sc = __builtin_amdgcn_exp2f(L.m - mb);
    L.Sb *= sc;
    L.S2b *= sc * sc;
    L.S *= (double)sc;
    L.S2 *= (double)sc * (double)sc;
#pragma unroll
    for (int d = 0; d < NM; ++d) L.g[d] *= sc;
    L.m = mb;
  }
}

template <int NM>
__device__ __forceinline__ void lse_flush(LseAcc<NM>& L) {
  L.S += (double)L.Sb;
  L.S2 += (double)L.S2b;
  L.Sb = L.S2b = 0.f;
}

template <int NM>
__device__ __forceinline__ void write_partials(const SweepArgs& A, const LseAcc<NM>& L, int64_t q, int split,
                                               bool with_z) {
  const int64_t sq = (int64_t)split * A.Q + q;
  A.part.m[sq] = L.m;
  A.part.S[sq] = L.S;
  A.part.S2[sq] = L.S2;
#pragma unroll
  for (int d = 0; d < NM; ++d) {
    if (d < A.n) {
      const int64_t idx = ((int64_t)split * A.n + d) * A.Q + q;
      A.part.G[idx] = L.g[d];
      if (with_z) A.part.Z[idx] = L.zs[d];
    }
  }
}

// ------------------------------------------------------------ common table (CRN)
// One block of the pair loop: queries qblock*QB .. +QB-1 (QB =
// kQueriesPerBlockValu, one per thread), sample split `split`.
template <int DATUM, int NM, int MP, bool BF16>
__device__ __forceinline__ void sweep_crn_block(const SweepArgs& A, int64_t qblock, int split) {
  constexpr int QB = kQueriesPerBlockValu;
  __shared__ float zs[NM][kBlk];
  const int64_t q = qblock * QB + threadIdx.x;
  const bool active = q < A.Q;
  const int64_t qs = active ? q : A.Q - 1;   // a valid state to read for idle lanes
  const int i_begin = split * A.ns;
  const int i_end = min(A.N, i_begin + A.ns);

  PairConst<DATUM, NM> P;
  pair_setup<DATUM, NM>(P, A, qs);
  LseAcc<NM> L;
  lse_init<NM>(L);

  for (int i0 = i_begin; i0 < i_end; i0 += kBlk) {
    const int cnt = min(kBlk, i_end - i0);
    for (int e = threadIdx.x; e < NM * kBlk; e += QB) {
      const int d = e / kBlk, j = e % kBlk;
      float z = 0.f;
      if (d < A.n && j < cnt) {
        const int64_t idx = (int64_t)d * A.tstride + i0 + j;
        if constexpr (BF16) z = bf16_to_f32(static_cast<const uint16_t*>(A.table)[idx]);
        else z = static_cast<const float*>(A.table)[idx];
      }
      zs[d][j] = z;
    }
    __syncthreads();
    // samples per max-rebase batch: fewer for wide states to bound registers
    constexpr int kB = NM >= 32 ? 4 : 8;
    for (int j0 = 0; j0 < cnt; j0 += kB) {
      float a[kB];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) {
        const int j = j0 + jj;
        const float w = pair_log2w<DATUM, NM, MP>(P, A.dp, [&](int d) { return zs[d][j]; });
        a[jj] = (j < cnt) ? w : -INFINITY;
      }
      float mb = a[0];
#pragma unroll
      for (int jj = 1; jj < kB; ++jj) mb = fmaxf(mb, a[jj]);
      lse_rebase<NM>(L, mb);
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) {
        const float w = __builtin_amdgcn_exp2f(a[jj] - L.m);
        L.Sb += w;
        L.S2b = fmaf(w, w, L.S2b);
#pragma unroll
        for (int d = 0; d < NM; ++d) L.g[d] = fmaf(w, zs[d][j0 + jj], L.g[d]);
      }
    }
    lse_flush<NM>(L);
    __syncthreads();
  }
  if (active) write_partials<NM>(A, L, q, split, false);
}

template <int DATUM, int NM, int MP, bool BF16>
__global__ __launch_bounds__(kQueriesPerBlockValu) void sweep_crn_kernel(SweepArgs A) {
  if (A.done && *A.done) return;
  sweep_crn_block<DATUM, NM, MP, BF16>(A, blockIdx.x, blockIdx.y);
}

// Many problems in one launch: block b serves work item items[b] =
// (problem, query block, sample split) with that problem's arguments.
template <int DATUM, int NM, int MP, bool BF16>
__global__ __launch_bounds__(kQueriesPerBlockValu) void sweep_crn_batched_kernel(const SweepArgs* probs, const int4* items,
                                                                     int count, int* counter) {
  __shared__ int slot;
  for (int b = counter ? next_item(counter, &slot) : (int)blockIdx.x; b < count;
       b = counter ? next_item(counter, &slot) : count) {
    const int4 it = work_item(items, b);
    const SweepArgs& A = problem_args(probs, it.x);
    if (A.done && *A.done) continue;
    sweep_crn_block<DATUM, NM, MP, BF16>(A, it.y, it.z);
  }
}

// ------------------------------------------------------------------ fresh draws
template <int DATUM, int NM, int MP, bool BF16>
__global__ __launch_bounds__(kThreads) void sweep_fresh_kernel(SweepArgs A) {
  if (A.done && *A.done) return;
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= A.Q) return;
  const int split = blockIdx.y;
  const int i_begin = split * A.ns;            // a multiple of 4
  const int i_end = min(A.N, i_begin + A.ns);

  PairConst<DATUM, NM> P;
  pair_setup<DATUM, NM>(P, A, q);
  LseAcc<NM> L;
  lse_init<NM>(L);
  const uint32_t stream = (uint32_t)q;

  int rounds = 0;
  for (int i0 = i_begin; i0 < i_end; i0 += 4) {
    float zr[NM][4];
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      if (d < A.n) {
        normals4((uint32_t)(i0 >> 2), (uint32_t)d, stream, A.tag, A.k0, A.k1, zr[d]);
        if constexpr (BF16) {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) zr[d][jj] = round_bf16(zr[d][jj]);
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) zr[d][jj] = 0.f;
      }
    }
    float a[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const float w = pair_log2w<DATUM, NM, MP>(P, A.dp, [&](int d) { return zr[d][jj]; });
      a[jj] = (i0 + jj < i_end) ? w : -INFINITY;
    }
    const float mb = fmaxf(fmaxf(a[0], a[1]), fmaxf(a[2], a[3]));
    lse_rebase<NM>(L, mb);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const bool valid = i0 + jj < i_end;
      const float w = __builtin_amdgcn_exp2f(a[jj] - L.m);
      L.Sb += w;
      L.S2b = fmaf(w, w, L.S2b);
#pragma unroll
      for (int d = 0; d < NM; ++d) {
        L.g[d] = fmaf(w, zr[d][jj], L.g[d]);
        if (A.cv && valid) L.zs[d] += zr[d][jj];
      }
    }
    if (++rounds == kBlk / 4) { lse_flush<NM>(L); rounds = 0; }
  }
  lse_flush<NM>(L);
  write_partials<NM>(A, L, q, split, A.cv != 0);
}

// Grid of a batched launch: one block per item, or for a persistent launch
// the blocks the device holds at once (never more than the items).
template <class Kernel>
unsigned batch_grid(Kernel kernel, int threads, const SweepBatch* b) {
  if (!b->counter) return (unsigned)b->count;
  int dev = 0, cus = 1, per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return (unsigned)b->count;
  return (unsigned)std::max(1, std::min(b->count, cus * std::max(per_cu, 1)));
}

template <int DATUM, int NM, int MP>
hipError_t launch_sweep_dn(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  if (a.mfma) {
    if constexpr (NM >= 16 && DATUM == HJG_L_MIN_PAIR_DISKS) {
      if (fresh || !bf16) return hipErrorInvalidValue;
      if (b) {
        const unsigned g = batch_grid(sweep_pairs_batched_kernel<NM, MP>, kPThreads, b);
        sweep_pairs_batched_kernel<NM, MP><<<g, kPThreads, 0, s>>>(b->probs, b->items, b->count, b->counter);
      } else {
        const dim3 grid((unsigned)((a.Q + kPQ - 1) / kPQ), (unsigned)a.splits);
        sweep_pairs_kernel<NM, MP><<<grid, kPThreads, 0, s>>>(a);
      }
      return hipGetLastError();
    } else if constexpr (NM >= 16 && DATUM != HJG_L_KNN_BALLS && DATUM != HJG_L_DISC_UNION) {
      if (fresh || !bf16) return hipErrorInvalidValue;
      if (b) {
        const unsigned g = batch_grid(sweep_mfma_batched_kernel<DATUM, NM, MP>, 256, b);
        sweep_mfma_batched_kernel<DATUM, NM, MP><<<g, 256, 0, s>>>(b->probs, b->items, b->count, b->counter);
      } else {
        const dim3 grid((unsigned)((a.Q + kMQ - 1) / kMQ), (unsigned)a.splits);
        sweep_mfma_kernel<DATUM, NM, MP><<<grid, 256, 0, s>>>(a);
      }
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (b) {
    if (fresh) return hipErrorInvalidValue;
    if (bf16) {
      const unsigned g = batch_grid(sweep_crn_batched_kernel<DATUM, NM, MP, true>, kQueriesPerBlockValu, b);
      sweep_crn_batched_kernel<DATUM, NM, MP, true><<<g, kQueriesPerBlockValu, 0, s>>>(b->probs, b->items, b->count, b->counter);
    } else {
      const unsigned g = batch_grid(sweep_crn_batched_kernel<DATUM, NM, MP, false>, kQueriesPerBlockValu, b);
      sweep_crn_batched_kernel<DATUM, NM, MP, false><<<g, kQueriesPerBlockValu, 0, s>>>(b->probs, b->items, b->count, b->counter);
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((a.Q + kThreads - 1) / kThreads), (unsigned)a.splits);
  if (fresh) {
    if constexpr (NM <= 16) {
      if (bf16) sweep_fresh_kernel<DATUM, NM, MP, true><<<grid, kThreads, 0, s>>>(a);
      else sweep_fresh_kernel<DATUM, NM, MP, false><<<grid, kThreads, 0, s>>>(a);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    constexpr int QB = kQueriesPerBlockValu;
    const dim3 gridc((unsigned)((a.Q + QB - 1) / QB), (unsigned)a.splits);
    if (bf16) sweep_crn_kernel<DATUM, NM, MP, true><<<gridc, QB, 0, s>>>(a);
    else sweep_crn_kernel<DATUM, NM, MP, false><<<gridc, QB, 0, s>>>(a);
  }
  return hipGetLastError();
}

// Disc pairs: the exact pair count as a template argument for the sizes the
// workloads use, otherwise the bucket's NM/3 pairs with padded pairs far away.
template <int NM, int M>
hipError_t launch_pairs_exact(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_dn<HJG_L_MIN_PAIR_DISKS, NM, M>(a, fresh, bf16, s, b);
}

template <int NM, int M>
hipError_t launch_capture_exact(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  return launch_sweep_dn<HJG_L_CAPTURE, NM, M>(a, fresh, bf16, s, b);
}

template <int DATUM>
hipError_t launch_sweep_d(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  if constexpr (DATUM == HJG_L_CAPTURE) {
    switch (a.n / 3) {
      case 2: return launch_capture_exact<8, 2>(a, fresh, bf16, s, b);
      case 3: return launch_capture_exact<16, 3>(a, fresh, bf16, s, b);
      case 4: return launch_capture_exact<16, 4>(a, fresh, bf16, s, b);
      case 5: return launch_capture_exact<16, 5>(a, fresh, bf16, s, b);
      case 6: return launch_capture_exact<32, 6>(a, fresh, bf16, s, b);
      case 7: return launch_capture_exact<32, 7>(a, fresh, bf16, s, b);
      case 8: return launch_capture_exact<32, 8>(a, fresh, bf16, s, b);
      case 9: return launch_capture_exact<32, 9>(a, fresh, bf16, s, b);
      case 10: return launch_capture_exact<32, 10>(a, fresh, bf16, s, b);
      case 11: return launch_capture_exact<48, 11>(a, fresh, bf16, s, b);
      case 12: return launch_capture_exact<48, 12>(a, fresh, bf16, s, b);
      case 13: return launch_capture_exact<48, 13>(a, fresh, bf16, s, b);
      case 14: return launch_capture_exact<48, 14>(a, fresh, bf16, s, b);
      case 15: return launch_capture_exact<48, 15>(a, fresh, bf16, s, b);
      case 16: return launch_capture_exact<48, 16>(a, fresh, bf16, s, b);
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (DATUM == HJG_L_KNN_BALLS) {
    return launch_sweep_dn<DATUM, 8, 0>(a, fresh, bf16, s, b);
  } else if constexpr (DATUM == HJG_L_DISC_UNION) {
    switch (n_bucket(a.n)) {
      case 4: return launch_sweep_dn<DATUM, 4, 0>(a, fresh, bf16, s, b);
      case 8: return launch_sweep_dn<DATUM, 8, 0>(a, fresh, bf16, s, b);
      case 16: return launch_sweep_dn<DATUM, 16, 0>(a, fresh, bf16, s, b);
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (DATUM == HJG_L_MIN_PAIR_DISKS) {
    switch (a.n / 3) {
      case 1: return launch_pairs_exact<4, 1>(a, fresh, bf16, s, b);
      case 2: return launch_pairs_exact<8, 2>(a, fresh, bf16, s, b);
      case 3: return launch_pairs_exact<16, 3>(a, fresh, bf16, s, b);
      case 4: return launch_pairs_exact<16, 4>(a, fresh, bf16, s, b);
      case 5: return launch_pairs_exact<16, 5>(a, fresh, bf16, s, b);
      case 6: return launch_pairs_exact<32, 6>(a, fresh, bf16, s, b);
      case 7: return launch_pairs_exact<32, 7>(a, fresh, bf16, s, b);
      case 8: return launch_pairs_exact<32, 8>(a, fresh, bf16, s, b);
      case 9: return launch_pairs_exact<32, 9>(a, fresh, bf16, s, b);
      case 10: return launch_pairs_exact<32, 10>(a, fresh, bf16, s, b);
      case 11: return launch_pairs_exact<48, 11>(a, fresh, bf16, s, b);
      case 12: return launch_pairs_exact<48, 12>(a, fresh, bf16, s, b);
      case 13: return launch_pairs_exact<48, 13>(a, fresh, bf16, s, b);
      case 14: return launch_pairs_exact<48, 14>(a, fresh, bf16, s, b);
      case 15: return launch_pairs_exact<48, 15>(a, fresh, bf16, s, b);
      default: return launch_pairs_exact<48, 16>(a, fresh, bf16, s, b);
    }
  } else {
    switch (n_bucket(a.n)) {
      case 4: return launch_sweep_dn<DATUM, 4, 0>(a, fresh, bf16, s, b);
      case 8: return launch_sweep_dn<DATUM, 8, 0>(a, fresh, bf16, s, b);
      case 16: return launch_sweep_dn<DATUM, 16, 0>(a, fresh, bf16, s, b);
      case 32: return launch_sweep_dn<DATUM, 32, 0>(a, fresh, bf16, s, b);
      default: return launch_sweep_dn<DATUM, 48, 0>(a, fresh, bf16, s, b);
    }
  }
}

}  // namespace hjg
