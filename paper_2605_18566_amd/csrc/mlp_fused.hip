// The surrogate network's fused training step (two launches per step); see
// mlp_fused.h for the division of the work.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "mlp_fused.h"

namespace hjg {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int R = kFusedRows;

// logistic function with the hardware reciprocal (as every network kernel)
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Shapes of one product of the rows kernel: out[16][N] = src[16][K] W^T.
// The wave owns the 16-column tiles wave, wave + 4, ... (NT < 4: waves
// beyond NT repeat tile wave % NT and store nothing).
template <int K, int N>
struct PhaseShape {
  static constexpr int NT = N / 16, TW = NT >= 4 ? NT / 4 : 1, KSP = K / 32;
  static_assert(N % 16 == 0 && K % 32 == 0 && (NT < 4 || NT % 4 == 0), "phase shape");
};

template <int K, int N>
using PhaseW = bf16x8[PhaseShape<K, N>::TW][PhaseShape<K, N>::KSP];

// Operand lanes of v_mfma_f32_16x16x32_bf16: A[i = l%16][k = 8(l/16)..+7],
// B[k = 8(l/16)..+7][j = l%16]; result lane l holds rows 4(l/16)..+3 of
// column l%16.  Every load and product of a phase is unconditional, so the
// weights of the next phase stay in flight while this phase computes.
template <int K, int N>
__device__ __forceinline__ void load_phase(const __bf16* W, int wave, int lane, PhaseW<K, N>& w) {
  using S = PhaseShape<K, N>;
#pragma unroll
  for (int j = 0; j < S::TW; ++j) {
    const int t = S::NT >= 4 ? wave + 4 * j : wave % S::NT;
    const __bf16* row = W + (int64_t)(16 * t + (lane & 15)) * K + 8 * (lane >> 4);
#pragma unroll
    for (int ks = 0; ks < S::KSP; ++ks) w[j][ks] = *reinterpret_cast<const bf16x8*>(row + 32 * ks);
  }
}

}  // namespace

// Rows kernel for a network of hidden width W, padded input IN, padded output
// OUT and D hidden layers: phases 0..D forward (D hidden, then the output with
// the loss), then D backward products (errors of hidden layers D-1 .. 0).
template <int W, int IN, int OUT, int D>
__global__ __launch_bounds__(256) void fused_rows_kernel(FusedRowsArgs a) {
  constexpr int WX = W > IN ? (W > OUT ? W : OUT) : (IN > OUT ? IN : OUT);
  constexpr int LH = WX + 8;
  __shared__ __attribute__((aligned(16))) __bf16 hbuf[2][R][LH];
  __shared__ float zs[D][R][W];
  __shared__ float bias[D + 1][WX];
  __shared__ float tgt[R][OUT];
  __shared__ float lws[OUT];
  __shared__ int srow[R];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.x * R;
  const int64_t bidx = a.batch ? *a.batch : 0;
  if (tid < R) srow[tid] = a.perm ? a.perm[bidx * a.B + r0 + tid] : r0 + tid;
#pragma unroll
  for (int l = 0; l <= D; ++l) {
    const int nl = l < D ? W : OUT;
    for (int c = tid; c < nl; c += 256) bias[l][c] = a.ph[l].bias[c];
  }
  for (int c = tid; c < OUT; c += 256) lws[c] = c < a.nout ? a.lw[c] : 0.f;
  __syncthreads();
  for (int e = tid; e < R * (IN / 8); e += 256) {
    const int r = e / (IN / 8), c = (e % (IN / 8)) * 8;
    *reinterpret_cast<bf16x8*>(&hbuf[0][r][c]) = *reinterpret_cast<const bf16x8*>(a.X + (int64_t)srow[r] * IN + c);
  }
  for (int e = tid; e < R * OUT; e += 256) {
    const int r = e / OUT, c = e % OUT;
    tgt[r][c] = a.T[(int64_t)srow[r] * OUT + c];
  }
  __syncthreads();
  for (int c = tid; c < IN; c += 256) {
    bf16x8 lo, hi;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      lo[r] = hbuf[0][r][c];
      hi[r] = hbuf[0][8 + r][c];
    }
    *reinterpret_cast<bf16x8*>(a.X0T + (int64_t)c * a.B + r0) = lo;
    *reinterpret_cast<bf16x8*>(a.X0T + (int64_t)c * a.B + r0 + 8) = hi;
  }

  double loss = 0.0;
  const int rb = 4 * (lane >> 4);
  // product of phase PH (compile time) from hbuf[PH % 2] into hbuf[1 - PH % 2]
  auto run = [&](auto ph, auto& w) {
    constexpr int PHI = decltype(ph)::value;
    constexpr bool FWD = PHI <= D;
    constexpr int L = FWD ? PHI : 2 * D + 1 - PHI;               // layer of the product
    constexpr int K = FWD ? (L == 0 ? IN : W) : (L == D ? OUT : W);
    constexpr int N = FWD ? (L == D ? OUT : W) : W;
    constexpr int KIND = FWD ? (L < D ? PH_FWD_HIDDEN : PH_FWD_OUT) : PH_BWD;
    constexpr int S = PHI % 2;
    using SH = PhaseShape<K, N>;
    const FusedPhase& P = a.ph[PHI];
    f32x4 acc[SH::TW];
#pragma unroll
    for (int j = 0; j < SH::TW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < SH::KSP; ++ks) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&hbuf[S][lane & 15][32 * ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < SH::TW; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w[j][ks], acc[j], 0, 0, 0);
    }
    const bool owner = SH::NT >= 4 || wave < SH::NT;
#pragma unroll
    for (int j = 0; j < SH::TW; ++j) {
      const int t = SH::NT >= 4 ? wave + 4 * j : wave % SH::NT;
      const int col = 16 * t + (lane & 15);
      bf16x4 o;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rb + v;
        __bf16 hv;
        if constexpr (KIND == PH_FWD_HIDDEN) {
          const float z = acc[j][v] + bias[L][col];
          zs[L][row][col] = z;
          hv = (__bf16)(z * sigm(z));
        } else if constexpr (KIND == PH_FWD_OUT) {
          const float y = acc[j][v] + bias[L][col];
          const float diff = y - tgt[row][col];
          // padded columns carry a zero weight: no loss and no error
          if (owner) loss += (double)lws[col] * (double)diff * (double)diff;
          hv = (__bf16)(2.0f * lws[col] * diff / (float)a.B);
        } else {
          const float z = zs[L - 1][row][col];
          const float sg = sigm(z);
          hv = (__bf16)(acc[j][v] * sg * (1.0f + z * (1.0f - sg)));
        }
        if (owner) hbuf[1 - S][row][col] = hv;
        o[v] = hv;
      }
      if (owner) *reinterpret_cast<bf16x4*>(P.outT + (int64_t)col * a.B + r0 + rb) = o;
    }
    __syncthreads();
  };
  // phases in order, the next phase's weights requested before each product
  constexpr int NPH = 2 * D + 1;
  auto step = [&](auto ph, auto& wcur, auto& self) {
    constexpr int PHI = decltype(ph)::value;
    if constexpr (PHI + 1 < NPH) {
      constexpr int PN = PHI + 1;
      constexpr bool FN = PN <= D;
      constexpr int LN = FN ? PN : 2 * D + 1 - PN;
      constexpr int KN = FN ? (LN == 0 ? IN : W) : (LN == D ? OUT : W);
      constexpr int NN = FN ? (LN == D ? OUT : W) : W;
      PhaseW<KN, NN> wn;
      load_phase<KN, NN>(a.ph[PN].W, wave, lane, wn);
      run(ph, wcur);
      self(std::integral_constant<int, PN>{}, wn, self);
    } else {
      run(ph, wcur);
    }
  };
  PhaseW<IN, W> w0;
  load_phase<IN, W>(a.ph[0].W, wave, lane, w0);
  step(std::integral_constant<int, 0>{}, w0, step);
  // ---- the block's loss (fixed order)
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
  if (lane == 0) red[wave] = loss;
  __syncthreads();
  if (tid == 0) a.block_loss[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One 32 x 32 tile of one layer's weight gradient: dW[m][n] = sum_b dz^T[m][b] h^T[n][b].
// Operand lanes of v_mfma_f32_32x32x16_bf16: A[i = l%32][k = 8(l/32)..+7],
// B[k = 8(l/32)..+7][j = l%32]; result lane l holds rows 8(v/4) + 4(l/32) + v%4
// of column l%32.  The four waves take a quarter of the batch each; the
// operands of 16 k-steps are requested before their products (and the next
// 16 before those products run).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void fused_weights_kernel(
    FusedWeightsArgs a) {
  __shared__ float part[4][16][64];
  __shared__ float rpart[4][64];
  __shared__ float sched[3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x;
  int l = 0;
  while (l + 1 < a.L && b >= a.layer[l + 1].first) ++l;
  const FusedLayer& Y = a.layer[l];
  const int t = b - Y.first;
  const int m0 = 32 * (t / Y.tiles_n), n0 = 32 * (t % Y.tiles_n);
  const bool rowsum = n0 == 0;
  const int kw = a.B / 4, kb = wave * kw;
  const __bf16* arow = Y.A + (int64_t)(m0 + (lane & 31)) * a.B + kb + 8 * (lane >> 5);
  const __bf16* brow = Y.Bm + (int64_t)(n0 + (lane & 31)) * a.B + kb + 8 * (lane >> 5);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float rs = 0.f;
  constexpr int CH = 16;   // k-steps per chunk
  const int nst = kw / 16;
  bf16x8 av[2][CH], bv[2][CH];
  auto load = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int st = c * CH + i;
      if (st < nst) {
        av[buf][i] = *reinterpret_cast<const bf16x8*>(arow + 16 * st);
        bv[buf][i] = *reinterpret_cast<const bf16x8*>(brow + 16 * st);
      }
    }
  };
  auto compute = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (c * CH + i < nst) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[buf][i], bv[buf][i], acc, 0, 0, 0);
        if (rowsum) {
#pragma unroll
          for (int e = 0; e < 8; ++e) rs += (float)av[buf][i][e];
        }
      }
    }
  };
  const int nch = (nst + CH - 1) / CH;
  load(0, 0);
  for (int c = 0; c < nch; c += 2) {
    if (c + 1 < nch) load(c + 1, 1);
    compute(c, 0);
    if (c + 1 < nch) {
      if (c + 2 < nch) load(c + 2, 0);
      compute(c + 1, 1);
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) part[wave][v][lane] = acc[v];
  if (rowsum) rpart[wave][lane] = rs;
  if (tid == 0 && a.adam) {
    const double k = (double)a.ctr[0], step = (double)(a.ctr[1] + 1);
    sched[0] = (float)(a.lr_min + 0.5 * (a.lr_max - a.lr_min) * (1.0 + cos(M_PI * k / (double)a.total)));
    sched[1] = (float)(1.0 - pow((double)a.b1, step));
    sched[2] = (float)(1.0 - pow((double)a.b2, step));
  }
  __syncthreads();
  const float lr = a.adam ? sched[0] : 0.f, bc1 = a.adam ? sched[1] : 1.f, bc2 = a.adam ? sched[2] : 1.f;
  auto update = [&](int64_t idx, float gi) -> float {
    const float mi = a.b1 * a.m[idx] + (1.0f - a.b1) * gi;
    const float vi = a.b2 * a.v[idx] + (1.0f - a.b2) * gi * gi;
    a.m[idx] = mi;
    a.v[idx] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    const float wi = a.w[idx] - lr * (mh / (sqrtf(vh) + a.eps) + a.wd * a.w[idx]);
    a.w[idx] = wi;
    return wi;
  };
  // the tile's 1,024 sums, four per thread, the waves added in order
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = 4 * tid + q;
    const int v = e / 64, ln = e % 64;
    const float gsum = ((part[0][v][ln] + part[1][v][ln]) + part[2][v][ln]) + part[3][v][ln];
    const int m = m0 + 8 * (v / 4) + 4 * (ln >> 5) + (v % 4), n = n0 + (ln & 31);
    const int64_t idx = Y.woff + (int64_t)m * Y.fin + n;
    if (a.adam) {
      const __bf16 wb = (__bf16)update(idx, gsum);
      Y.Wb[(int64_t)m * Y.fin + n] = wb;
      Y.WbT[(int64_t)n * Y.fout + m] = wb;
    } else {
      a.g[idx] = gsum;
    }
  }
  if (rowsum && tid < 32) {
    float gsum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) gsum += rpart[w][tid] + rpart[w][tid + 32];
    const int64_t idx = Y.boff + m0 + tid;
    if (a.adam) (void)update(idx, gsum);
    else a.g[idx] = gsum;
  }
  if (b == 0 && tid == 0 && a.acc) {
    double s = 0.0;
    for (int i = 0; i < a.nbl; ++i) s += a.block_loss[i];
    a.acc[0] += s;
  }
  // the last block to finish advances the step counters for the next step
  if (a.ticket) {
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const int done = atomicAdd(a.ticket, 1);
      if (done == (int)gridDim.x - 1) {
        int64_t* ctr = const_cast<int64_t*>(a.ctr);
        ctr[0] += 1;
        ctr[1] += 1;
        ctr[2] += 1;
        *a.ticket = 0;
        __threadfence();
      }
    }
  }
}

namespace {

template <int W, int P, int D>
hipError_t rows_launch(const FusedRowsArgs& a, hipStream_t s) {
  fused_rows_kernel<W, P, P, D><<<a.B / R, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int W, int P>
hipError_t rows_by_depth(const FusedRowsArgs& a, int D, hipStream_t s) {
  switch (D) {
    case 2: return rows_launch<W, P, 2>(a, s);
    case 3: return rows_launch<W, P, 3>(a, s);
    case 4: return rows_launch<W, P, 4>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int W>
hipError_t rows_by_pad(const FusedRowsArgs& a, int D, hipStream_t s) {
  switch (a.in_p) {
    case 32: return rows_by_depth<W, 32>(a, D, s);
    case 64: return rows_by_depth<W, 64>(a, D, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool fused_rows_supported(int width, int in_p, int out_p, int depth) {
  return (width == 64 || width == 128 || width == 256) && (in_p == 32 || in_p == 64) && out_p == in_p && depth >= 2 &&
         depth <= kFusedMaxHidden;
}

hipError_t launch_fused_rows(const FusedRowsArgs& a, int width, int depth, hipStream_t s) {
  if (!fused_rows_supported(width, a.in_p, a.out_p, depth)) return hipErrorInvalidValue;
  switch (width) {
    case 64: return rows_by_pad<64>(a, depth, s);
    case 128: return rows_by_pad<128>(a, depth, s);
    case 256: return rows_by_pad<256>(a, depth, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fused_weights(const FusedWeightsArgs& a, hipStream_t s) {
  fused_weights_kernel<<<a.tiles, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace hjg
