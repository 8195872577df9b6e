// Per-query kernels around the pair loop: draw tables, Picard initialisation,
// the float64 merge of sample splits with the estimator formulas, the Picard
// update of coefficient and shift, and the residual reduction.
#include <algorithm>

#include "kernels.h"

namespace hjg {

hipError_t launch_sweep_half_sqnorm(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_ball(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_min_pair_disks(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_knn_balls(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_capture(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_disc_union(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);
hipError_t launch_sweep_linear(const SweepArgs&, int, int, hipStream_t, const SweepBatch*);

hipError_t launch_sweep(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b) {
  switch (a.dp.kind) {
    case HJG_L_HALF_SQNORM: return launch_sweep_half_sqnorm(a, fresh, bf16, s, b);
    case HJG_L_BALL: return launch_sweep_ball(a, fresh, bf16, s, b);
    case HJG_L_MIN_PAIR_DISKS: return launch_sweep_min_pair_disks(a, fresh, bf16, s, b);
    case HJG_L_KNN_BALLS: return launch_sweep_knn_balls(a, fresh, bf16, s, b);
    case HJG_L_CAPTURE: return launch_sweep_capture(a, fresh, bf16, s, b);
    case HJG_L_DISC_UNION: return launch_sweep_disc_union(a, fresh, bf16, s, b);
    case HJG_L_LINEAR: return launch_sweep_linear(a, fresh, bf16, s, b);
    default: return hipErrorInvalidValue;
  }
}

namespace {

constexpr uint32_t kCrnStream = 0xFFFFFFFFu;

// ------------------------------------------------------------------ draw table
// z[d][i] for d < n, i < limit, row stride tstride (>= limit).
__global__ __launch_bounds__(kThreads) void table_kernel(int n, int64_t limit, int64_t tstride, uint32_t k0,
                                                         uint32_t k1, uint32_t tag, int bf16, void* out) {
  const int64_t groups = (limit + 3) / 4;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= groups * n) return;
  const int d = (int)(idx / groups);
  const int64_t g = idx % groups;
  float z[4];
  normals4((uint32_t)g, (uint32_t)d, kCrnStream, tag, k0, k1, z);
  const int64_t base = (int64_t)d * tstride + 4 * g;
  if (bf16) {
    uint16_t* o = static_cast<uint16_t*>(out);
#pragma unroll
    for (int j = 0; j < 4; ++j) if (4 * g + j < limit) o[base + j] = f32_to_bf16_rne(z[j]);
  } else {
    float* o = static_cast<float*>(out);
#pragma unroll
    for (int j = 0; j < 4; ++j) if (4 * g + j < limit) o[base + j] = z[j];
  }
}

// zbar[d] = (1/N) sum_{i<N} z[d][i] in float64, one block per dimension,
// fixed reduction order (deterministic).
__global__ __launch_bounds__(kThreads) void zbar_kernel(int N, int64_t tstride, int bf16, const void* table,
                                                        double* zbar) {
  const int d = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const int64_t idx = (int64_t)d * tstride + i;
    s += bf16 ? (double)bf16_to_f32(static_cast<const uint16_t*>(table)[idx])
              : (double)static_cast<const float*>(table)[idx];
  }
  __shared__ double red[kThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) zbar[d] = red[0] / (double)N;
}

__global__ __launch_bounds__(kThreads) void philox_words_kernel(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2,
                                                                uint32_t c3, int64_t G, uint32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < G; g += stride) {
    const U4 w = philox4x32_10(U4{(uint32_t)g, c1, c2, c3}, k0, k1);
    out[4 * g + 0] = w.x;
    out[4 * g + 1] = w.y;
    out[4 * g + 2] = w.z;
    out[4 * g + 3] = w.w;
  }
}

__global__ __launch_bounds__(kThreads) void finite_kernel(const float* a, int64_t count, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) bad |= !isfinite(a[i]);
  if (bad) *flag = 1;   // benign race: every writer stores 1
}

// ------------------------------------------------------------ Picard start
template <int NM>
__device__ __forceinline__ void init_block(const InitArgs& I, int64_t qblock) {
  if (qblock == 0) {
    for (int k = threadIdx.x; k < I.K; k += kThreads) I.resid[k] = 0.0;
    if (threadIdx.x == 0) {
      *I.done = 0;
      *I.iters = 0;
      if (I.nonfinite) *I.nonfinite = 0;
    }
  }
  const int64_t q = qblock * kThreads + threadIdx.x;
  if (q >= I.Q) return;
  float x[NM], g[NM];
#pragma unroll
  for (int d = 0; d < NM; ++d) x[d] = d < I.n ? I.x[(int64_t)d * I.Q + q] : 0.f;
  const float l = datum_and_grad<NM>(I.dp, x, g, q, I.Q);
  I.vprev[q] = I.v0 ? I.v0[q] : l;                  // v^(0) = l(x), or the warm start
  if (I.p0) {
#pragma unroll
    for (int d = 0; d < NM; ++d) g[d] = d < I.n ? I.p0[(int64_t)d * I.Q + q] : 0.f;
  }
#pragma unroll
  for (int d = 0; d < NM; ++d) if (d < I.n) I.p[(int64_t)d * I.Q + q] = g[d];
  const float c = coefficient<NM>(I.hp, x, g);       // c^(0) from D l (or the warm start)
  I.c[q] = c;
  if (I.th) {
    const float s2c = -I.sigma * I.sigma * c;
#pragma unroll
    for (int d = 0; d < NM; ++d) if (d < I.n) I.th[(int64_t)d * I.Q + q] = s2c * g[d];
  }
}

template <int NM>
__global__ __launch_bounds__(kThreads) void init_kernel(InitArgs I) { init_block<NM>(I, blockIdx.x); }

template <int NM>
__global__ __launch_bounds__(kThreads) void init_batched_kernel(const InitArgs* args, const int2* items) {
  const int2 it = items[blockIdx.x];
  const InitArgs I = args[it.x];
  init_block<NM>(I, it.y);
}

// ------------------------------------------------------------ finalize
// Merge the split partials in float64 (max-rescaled sums), then
//   v = -(m ln 2 + ln(S/N)) / c,  Dv = -(theta + sigma (G/S - [zbar])) / (c sigma^2),
//   ESS = S^2 / S2,
// and, inside the Picard loop, the residual terms, the per-query flag and the
// next coefficient and shift from p = Dv.
// MERGE: several sample splits, merged in one pass (below); otherwise one
// split, whose sums need no rescaling and whose per-dimension loads go one at
// a time — the low register count keeps enough waves resident at large Q.
// Both forms give the same bits for one split (the rescale factor is exactly 1).
template <int NM, bool MERGE>
__device__ __forceinline__ void finalize_block(const FinalizeArgs& F, int64_t qblock) {
  const int64_t q = qblock * kThreads + threadIdx.x;
  const bool active = q < F.Q;
  double dv2 = 0.0, vp2 = 0.0, bad = 0.0;
  if (active) {
    const int64_t Q = F.Q;
    // One pass over the splits: each split's rescale factor is formed once
    // and applied to S, S2 and every gradient sum (each sum still runs over
    // the splits in ascending order).  Every per-dimension load is issued
    // without a branch (rows d >= n re-read row n - 1 and are never used), so
    // a split's loads are in flight together instead of one latency each.
    // Fresh draws (the only user of the per-query z sums) exist for n <= 16.
    constexpr bool kZ = NM <= 16;
    constexpr int NG = MERGE ? NM : 1;
    const bool zsum = kZ && F.cv && F.fresh;
    double M, S = 0.0, S2 = 0.0, G[NG], Z[MERGE && kZ ? NM : 1];
    float xv[NG], thv[NG];
    if constexpr (MERGE) {
      M = -INFINITY;
#pragma unroll 8
      for (int s = 0; s < F.splits; ++s) M = fmax(M, (double)F.part.m[(int64_t)s * Q + q]);
#pragma unroll
      for (int d = 0; d < NM; ++d) G[d] = 0.0;
#pragma unroll
      for (int d = 0; d < (kZ ? NM : 1); ++d) Z[d] = 0.0;
      for (int s = 0; s < F.splits; ++s) {
        const double f = exp2((double)F.part.m[(int64_t)s * Q + q] - M);
        S += F.part.S[(int64_t)s * Q + q] * f;
        S2 += F.part.S2[(int64_t)s * Q + q] * f * f;
#pragma unroll
        for (int d = 0; d < NM; ++d) {
          const int64_t idx = ((int64_t)s * F.n + (d < F.n ? d : F.n - 1)) * Q + q;
          G[d] += (double)F.part.G[idx] * f;
        }
        if constexpr (kZ) {
          if (zsum) {
#pragma unroll
            for (int d = 0; d < NM; ++d) Z[d] += (double)F.part.Z[((int64_t)s * F.n + (d < F.n ? d : F.n - 1)) * Q + q];
          }
        }
      }
#pragma unroll
      for (int d = 0; d < NM; ++d) {
        const int64_t idx = (int64_t)(d < F.n ? d : F.n - 1) * Q + q;
        xv[d] = F.x[idx];
        thv[d] = F.theta ? F.theta[idx] : 0.f;
      }
    } else {
      M = (double)F.part.m[q];
      S = F.part.S[q];
      S2 = F.part.S2[q];
    }
    const double c = (double)F.c[q];
    const double sg = (double)F.sigma;
    const double v = -(M * kLn2 + log(S / (double)F.N)) / c;
    float xq[NM], pg[NM];
    bool finite = isfinite(v);
#pragma unroll
    for (int d = 0; d < NM; ++d) {
      xq[d] = 0.f;
      pg[d] = 0.f;
      if (d < F.n) {
        double gbar, zs = 0.0, th;
        if constexpr (MERGE) {
          gbar = G[d] / S;
          if constexpr (kZ) zs = Z[d];
          th = (double)thv[d];
          xq[d] = xv[d];
        } else {
          const int64_t idx = (int64_t)d * Q + q;
          gbar = (double)F.part.G[idx] / S;
          if (zsum) zs = (double)F.part.Z[idx];
          th = F.theta ? (double)F.theta[idx] : 0.0;
          xq[d] = F.x[idx];
        }
        if (F.cv) gbar -= zsum ? zs / (double)F.N : F.zbar_tab[d];
        const double gr = -(th + sg * gbar) / (c * sg * sg);
        pg[d] = (float)gr;
        finite = finite && isfinite(pg[d]);
        F.grad[(int64_t)d * Q + q] = pg[d];
      }
    }
    const float vf = (float)v;
    finite = finite && isfinite(vf);
    F.v[q] = vf;
    if (F.ess) F.ess[q] = (float)(S * S / S2);
    if (F.picard) {
      const float vp = F.vprev[q];
      const float dv = vf - vp;
      dv2 = (double)dv * (double)dv;
      vp2 = (double)vp * (double)vp;
      bad = finite ? 0.0 : 1.0;
      // a relative change that is not <= tol (NaN included), or a non-finite
      // output, is not converged
      if (F.flags) F.flags[q] = (!((fabsf(dv) / fmaxf(fabsf(vp), F.vfloor)) <= F.tol) || !finite) ? 1 : 0;
      F.vprev[q] = vf;
      if (F.c_out) F.c_out[q] = F.c[q];
      const float cn = coefficient<NM>(F.hp, xq, pg);
      if (F.th_next) {
        const float s2c = -F.sigma * F.sigma * cn;
#pragma unroll
        for (int d = 0; d < NM; ++d) if (d < F.n) F.th_next[(int64_t)d * Q + q] = s2c * pg[d];
      }
      F.c_next[q] = cn;
    }
  }
  if (F.picard) {
    for (int off = 32; off > 0; off >>= 1) {
      dv2 += __shfl_down(dv2, off, 64);
      vp2 += __shfl_down(vp2, off, 64);
      bad += __shfl_down(bad, off, 64);
    }
    __shared__ double red[3][kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { red[0][wid] = dv2; red[1][wid] = vp2; red[2][wid] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0, c = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) { a += red[0][w]; b += red[1][w]; c += red[2][w]; }
      F.blockpart[3 * qblock] = a;
      F.blockpart[3 * qblock + 1] = b;
      F.blockpart[3 * qblock + 2] = c;
    }
  }
}

template <int NM, bool MERGE>
__global__ __launch_bounds__(kThreads) void finalize_kernel(FinalizeArgs F) {
  if (F.done && *F.done) return;
  finalize_block<NM, MERGE>(F, blockIdx.x);
}

template <int NM>
__global__ __launch_bounds__(kThreads) void finalize_batched_kernel(const FinalizeArgs* args, const int2* items) {
  const int2 it = items[blockIdx.x];
  const FinalizeArgs F = args[it.x];
  if (F.done && *F.done) return;
  finalize_block<NM, true>(F, it.y);
}

// Relative L2 change over all queries from the block partials (float64, fixed order).
__device__ __forceinline__ void reduce_block(const ReduceArgs& R) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < R.nblocks; i += kThreads) {
    a += R.blockpart[3 * i];
    b += R.blockpart[3 * i + 1];
    c += R.blockpart[3 * i + 2];
  }
  __shared__ double ra[kThreads], rb[kThreads], rc[kThreads];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      ra[threadIdx.x] += ra[threadIdx.x + off];
      rb[threadIdx.x] += rb[threadIdx.x + off];
      rc[threadIdx.x] += rc[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double num = sqrt(ra[0]), den = sqrt(rb[0]);
    const double r = den > 0.0 ? num / den : num;
    R.resid[R.k] = r;
    *R.iters = R.k + 1;
    // the count of the last executed iteration is what the caller reads
    if (R.nonfinite) *R.nonfinite = (int)rc[0];
    if (r < (double)R.tol) *R.done = 1;
  }
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(ReduceArgs R) {
  if (*R.done) return;
  reduce_block(R);
}

// One block per problem of the list; k overrides the level.
__global__ __launch_bounds__(kThreads) void reduce_batched_kernel(const ReduceArgs* args, const int* plist, int k) {
  ReduceArgs R = args[plist[blockIdx.x]];
  if (*R.done) return;
  R.k = k;
  reduce_block(R);
}

}  // namespace

hipError_t launch_table(int n, int64_t limit, int64_t tstride, uint32_t k0, uint32_t k1, uint32_t tag, int bf16,
                        void* out, hipStream_t s) {
  const int64_t work = ((limit + 3) / 4) * n;
  table_kernel<<<(unsigned)((work + kThreads - 1) / kThreads), kThreads, 0, s>>>(n, limit, tstride, k0, k1, tag,
                                                                                  bf16, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void pair_coords_kernel(int m, int N, int64_t tstride, const uint16_t* table,
                                                               int zs, float* zd) {
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (int64_t)N * zs) return;
  const int64_t i = idx / zs;
  const int s = (int)(idx % zs);
  zd[idx] = s < 2 * m ? bf16_to_f32(table[(int64_t)(3 * (s / 2) + s % 2) * tstride + i]) : 0.f;
}

hipError_t launch_pair_coords(int m, int N, int64_t tstride, const void* table_bf16, int zs, float* zd, hipStream_t s) {
  const int64_t work = (int64_t)N * zs;
  pair_coords_kernel<<<(unsigned)((work + kThreads - 1) / kThreads), kThreads, 0, s>>>(
      m, N, tstride, static_cast<const uint16_t*>(table_bf16), zs, zd);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void fill_ints_kernel(int* a, int64_t count, int value) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) a[i] = value;
}

hipError_t launch_fill_ints(int* a, int64_t count, int value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_ints_kernel<<<(unsigned)((count + kThreads - 1) / kThreads), kThreads, 0, s>>>(a, count, value);
  return hipGetLastError();
}

hipError_t launch_zbar(int n, int N, int64_t tstride, int bf16, const void* table, double* zbar, hipStream_t s) {
  zbar_kernel<<<n, kThreads, 0, s>>>(N, tstride, bf16, table, zbar);
  return hipGetLastError();
}

hipError_t launch_philox_words(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t G,
                               uint32_t* out, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((G + kThreads - 1) / kThreads, 65536);
  philox_words_kernel<<<(unsigned)std::max<int64_t>(blocks, 1), kThreads, 0, s>>>(k0, k1, c1, c2, c3, G, out);
  return hipGetLastError();
}

hipError_t launch_finite_check(const float* a, int64_t count, int* flag, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((count + kThreads - 1) / kThreads, 4096);
  finite_kernel<<<(unsigned)std::max<int64_t>(blocks, 1), kThreads, 0, s>>>(a, count, flag);
  return hipGetLastError();
}

template <int NM>
void init_launch(const InitArgs& a, hipStream_t s, const ItemBatch<InitArgs>* b) {
  if (b) {
    init_batched_kernel<NM><<<b->count, kThreads, 0, s>>>(b->args, b->items);
  } else {
    const dim3 grid((unsigned)std::max<int64_t>((a.Q + kThreads - 1) / kThreads, 1));
    init_kernel<NM><<<grid, kThreads, 0, s>>>(a);
  }
}

template <int NM>
void finalize_launch(const FinalizeArgs& a, hipStream_t s, const ItemBatch<FinalizeArgs>* b) {
  if (b) {
    finalize_batched_kernel<NM><<<b->count, kThreads, 0, s>>>(b->args, b->items);
  } else {
    const dim3 grid((unsigned)((a.Q + kThreads - 1) / kThreads));
    if (a.splits > 1) finalize_kernel<NM, true><<<grid, kThreads, 0, s>>>(a);
    else finalize_kernel<NM, false><<<grid, kThreads, 0, s>>>(a);
  }
}

hipError_t launch_init(const InitArgs& a, hipStream_t s, const ItemBatch<InitArgs>* b) {
  switch (n_bucket(a.n)) {
    case 4: init_launch<4>(a, s, b); break;
    case 8: init_launch<8>(a, s, b); break;
    case 16: init_launch<16>(a, s, b); break;
    case 32: init_launch<32>(a, s, b); break;
    default: init_launch<48>(a, s, b); break;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s, const ItemBatch<FinalizeArgs>* b) {
  switch (n_bucket(a.n)) {
    case 4: finalize_launch<4>(a, s, b); break;
    case 8: finalize_launch<8>(a, s, b); break;
    case 16: finalize_launch<16>(a, s, b); break;
    case 32: finalize_launch<32>(a, s, b); break;
    default: finalize_launch<48>(a, s, b); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  reduce_kernel<<<1, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_reduce_batched(const ReduceArgs* args, const int* plist, int count, int k, hipStream_t s) {
  reduce_batched_kernel<<<count, kThreads, 0, s>>>(args, plist, k);
  return hipGetLastError();
}

}  // namespace hjg
