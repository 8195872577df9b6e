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

// Shapes of one product of the rows kernel: out[16][N] = src[16][K] W^T over
// NW waves.  The wave owns the 16-column tiles wave, wave + NW, ... (NT < NW:
// waves beyond NT repeat tile wave % NT and store nothing).
template <int K, int N, int NW>
struct PhaseShape {
  static constexpr int NT = N / 16, TW = NT >= NW ? NT / NW : 1, KSP = K / 32;
  static_assert(N % 16 == 0 && K % 32 == 0 && (NT < NW || NT % NW == 0), "phase shape");
};

template <int K, int N, int NW>
using PhaseW = bf16x8[PhaseShape<K, N, NW>::TW][PhaseShape<K, N, NW>::KSP];

// Operand lanes of v_mfma_f32_16x16x32_bf16: A[i = l%16][k = 8(l/16)..+7],
// B[k = 8(l/16)..+7][j = l%16]; result lane l holds rows 4(l/16)..+3 of
// column l%16.  Every load and product of a phase is unconditional, so the
// weights of the next phase stay in flight while this phase computes.
template <int K, int N, int NW>
__device__ __forceinline__ void load_phase(const __bf16* W, int wave, int lane, PhaseW<K, N, NW>& w) {
  using S = PhaseShape<K, N, NW>;
#pragma unroll
  for (int j = 0; j < S::TW; ++j) {
    const int t = S::NT >= NW ? wave + NW * j : wave % S::NT;
    const __bf16* row = W + (int64_t)(16 * t + (lane & 15)) * K + 8 * (lane >> 4);
#pragma unroll
    for (int ks = 0; ks < S::KSP; ++ks) w[j][ks] = *reinterpret_cast<const bf16x8*>(row + 32 * ks);
  }
}

}  // namespace

// Rows kernel for a network of hidden width W, padded input IN, padded output
// OUT and D hidden layers, NW waves per block: phases 0..D forward (D hidden,
// then the output with the loss), then D backward products (errors of hidden
// layers D-1 .. 0).
template <int W, int IN, int OUT, int D, int NW>
__global__ __launch_bounds__(64 * NW) void fused_rows_kernel(FusedRowsArgs a) {
  constexpr int NTH = 64 * NW;
  constexpr int WX = W > IN ? (W > OUT ? W : OUT) : (IN > OUT ? IN : OUT);
  constexpr int LH = WX + 8;
  __shared__ __attribute__((aligned(16))) __bf16 hbuf[2][R][LH];
  __shared__ float zs[D][R][W];
  __shared__ float bias[D + 1][WX];
  __shared__ __attribute__((aligned(16))) float tgt[R][OUT];
  __shared__ float lws[OUT];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.x * R;
#pragma unroll
  for (int l = 0; l <= D; ++l) {
    const int nl = l < D ? W : OUT;
    for (int c = tid; c < nl; c += NTH) bias[l][c] = a.ph[l].bias[c];
  }
  for (int c = tid; c < OUT; c += NTH) lws[c] = c < a.nout ? a.lw[c] : 0.f;
  __syncthreads();
  const __bf16* xb = a.X + (a.row0 + r0) * IN;
  const float* tb = a.T + (a.row0 + r0) * OUT;
  for (int e = tid; e < R * (IN / 8); e += NTH) {
    const int r = e / (IN / 8), c = (e % (IN / 8)) * 8;
    *reinterpret_cast<bf16x8*>(&hbuf[0][r][c]) = *reinterpret_cast<const bf16x8*>(xb + r * IN + c);
  }
  for (int e = tid; e < R * (OUT / 4); e += NTH) {
    const int r = e / (OUT / 4), c = (e % (OUT / 4)) * 4;
    *reinterpret_cast<f32x4*>(&tgt[r][c]) = *reinterpret_cast<const f32x4*>(tb + r * OUT + c);
  }
  __syncthreads();
  for (int c = tid; c < IN; c += NTH) {
    bf16x8 lo, hi;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      lo[r] = hbuf[0][r][c];
      hi[r] = hbuf[0][8 + r][c];
    }
    __bf16* dst = a.X0T + (int64_t)(r0 >> 6) * (IN * 64) + c * 64 + (r0 & 63);
    *reinterpret_cast<bf16x8*>(dst) = lo;
    *reinterpret_cast<bf16x8*>(dst + 8) = hi;
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
    using SH = PhaseShape<K, N, NW>;
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
    const bool owner = SH::NT >= NW || wave < SH::NT;
#pragma unroll
    for (int j = 0; j < SH::TW; ++j) {
      const int t = SH::NT >= NW ? wave + NW * j : wave % SH::NT;
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
      if (owner) *reinterpret_cast<bf16x4*>(P.outT + (int64_t)(r0 >> 6) * (N * 64) + col * 64 + (r0 & 63) + rb) = o;
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
      PhaseW<KN, NN, NW> wn;
      load_phase<KN, NN, NW>(a.ph[PN].W, wave, lane, wn);
      // keep the requests ahead of this phase's products (the scheduler
      // would otherwise sink them into the freed registers of this phase)
      __builtin_amdgcn_sched_barrier(0);
      run(ph, wcur);
      self(std::integral_constant<int, PN>{}, wn, self);
    } else {
      run(ph, wcur);
    }
  };
  PhaseW<IN, W, NW> w0;
  load_phase<IN, W, NW>(a.ph[0].W, wave, lane, w0);
  step(std::integral_constant<int, 0>{}, w0, step);
  // ---- the block's loss (fixed order)
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
  if (lane == 0) red[wave] = loss;
  __syncthreads();
  if (tid == 0) {
    double sl = 0.0;
    for (int w = 0; w < NW; ++w) sl += red[w];
    a.block_loss[blockIdx.x] = sl;
  }
}

// One 32 x 32 tile of one layer's weight gradient: dW[m][n] = sum_b dz^T[m][b] h^T[n][b].
// Operand lanes of v_mfma_f32_32x32x16_bf16: A[i = l%32][k = 8(l/32)..+7],
// B[k = 8(l/32)..+7][j = l%32]; result lane l holds rows 8(v/4) + 4(l/32) + v%4
// of column l%32.  The NWV waves split the batch (NST k-steps of 16 each); the
// loop is unrolled at compile time, the operands of the next 8 k-steps
// requested before the products of the current 8.
// Consecutive blocks go to different XCDs (round robin), so tiles are
// assigned in contiguous ranges per XCD: the tiles of one range share their
// row blocks of dz^T in that XCD's L2.
template <int NST, int NWV>
__global__ __launch_bounds__(64 * NWV) void fused_weights_kernel(FusedWeightsArgs a) {
  constexpr int CH = NST < 8 ? NST : 8;     // k-steps per chunk
  constexpr int NCH = NST / CH;
  static_assert(NST % CH == 0, "k-steps per wave");
  __shared__ float part[NWV][16][64];
  __shared__ float rpart[NWV][64];
  __shared__ float sched[3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nx = 8, q8 = a.tiles / nx, r8 = a.tiles % nx, x = blockIdx.x % nx;
  const int b = x * q8 + (x < r8 ? x : r8) + (int)blockIdx.x / nx;
  int l = 0;
  while (l + 1 < a.L && b >= a.layer[l + 1].first) ++l;
  const FusedLayer& Y = a.layer[l];
  const int t = b - Y.first;
  const int m0 = 32 * (t / Y.tiles_n), n0 = 32 * (t % Y.tiles_n);
  const int kb = wave * (16 * NST);
  const int h8 = 8 * (lane >> 5);
  const __bf16* abase = Y.A + (m0 + (lane & 31)) * 64;
  const __bf16* bbase = Y.Bm + (n0 + (lane & 31)) * 64;
  const int64_t fa = (int64_t)Y.fout * 64, fb = (int64_t)Y.fin * 64;
  // operands of k-step st: batch columns kb + 16 st + h8 .. + 7 (one 64-column block)
  auto aptr = [&](int st) {
    const int k = kb + 16 * st + h8;
    return reinterpret_cast<const bf16x8*>(abase + (k >> 6) * fa + (k & 63));
  };
  auto bptr = [&](int st) {
    const int k = kb + 16 * st + h8;
    return reinterpret_cast<const bf16x8*>(bbase + (k >> 6) * fb + (k & 63));
  };
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  float rs = 0.f;
  bf16x8 av[2][CH], bv[2][CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    av[0][i] = *aptr(i);
    bv[0][i] = *bptr(i);
  }
  // the epilogue's operands, requested now so that they arrive during the
  // products: this step's schedule, the thread's parameters and moments
  // (column n0 + tid % 32, rows m0 + 4 (tid / 32) .. + 3), the bias entries,
  // the rows kernel's loss sums
  const float sch = a.adam && tid < 3 ? a.sched[tid] : 0.f;
  const int n = n0 + (tid & 31), mr = m0 + 4 * (tid >> 5);
  const bool bias_row = n0 == 0 && tid < 32;
  float wq[4], mq[4], vq[4], wbias = 0.f, mbias = 0.f, vbias = 0.f;
  if (a.adam && tid < 256) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t idx = Y.woff + (int64_t)(mr + q) * Y.fin + n;
      wq[q] = a.w[idx];
      mq[q] = a.m[idx];
      vq[q] = a.v[idx];
    }
  }
  if (a.adam && bias_row) {
    wbias = a.w[Y.boff + m0 + tid];
    mbias = a.m[Y.boff + m0 + tid];
    vbias = a.v[Y.boff + m0 + tid];
  }
  const bool loss_wave = blockIdx.x == 0 && wave == 0 && a.acc;
  double blv[4] = {0.0, 0.0, 0.0, 0.0};
  if (loss_wave) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (lane + 64 * j < a.nbl) blv[j] = a.block_loss[lane + 64 * j];
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int cur = c & 1;
    if (c + 1 < NCH) {
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        av[1 - cur][i] = *aptr((c + 1) * CH + i);
        bv[1 - cur][i] = *bptr((c + 1) * CH + i);
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // the next chunk's requests stay ahead of these products
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[cur][i], bv[cur][i], acc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 8; ++e) rs += (float)av[cur][i][e];
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) part[wave][v][lane] = acc[v];
  rpart[wave][lane] = rs;
  if (tid < 3) sched[tid] = sch;
  __syncthreads();
  const float lr = a.adam ? sched[0] : 0.f, bc1 = a.adam ? sched[1] : 1.f, bc2 = a.adam ? sched[2] : 1.f;
  auto update = [&](int64_t idx, float gi, float wo, float mo, float vo) -> float {
    const float mi = a.b1 * mo + (1.0f - a.b1) * gi;
    const float vi = a.b2 * vo + (1.0f - a.b2) * gi * gi;
    a.m[idx] = mi;
    a.v[idx] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    const float wi = wo - lr * (mh / (sqrtf(vh) + a.eps) + a.wd * wo);
    a.w[idx] = wi;
    return wi;
  };
  // the thread's entries are 4 (tid / 64) + q of lane tid % 64 in every
  // wave's result
  bf16x4 wt;
  if (tid < 256) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int v = 4 * (tid >> 6) + q;
      float gsum = part[0][v][lane];
#pragma unroll
      for (int w = 1; w < NWV; ++w) gsum += part[w][v][lane];
      const int64_t idx = Y.woff + (int64_t)(mr + q) * Y.fin + n;
      if (a.adam) {
        const __bf16 wb = (__bf16)update(idx, gsum, wq[q], mq[q], vq[q]);
        Y.Wb[(int64_t)(mr + q) * Y.fin + n] = wb;
        wt[q] = wb;
      } else {
        a.g[idx] = gsum;
      }
    }
    if (a.adam) *reinterpret_cast<bf16x4*>(Y.WbT + (int64_t)n * Y.fout + mr) = wt;
  }
  if (bias_row) {
    float gsum = 0.f;
#pragma unroll
    for (int w = 0; w < NWV; ++w) gsum += rpart[w][tid] + rpart[w][tid + 32];
    const int64_t idx = Y.boff + m0 + tid;
    if (a.adam) (void)update(idx, gsum, wbias, mbias, vbias);
    else a.g[idx] = gsum;
  }
  // the step's loss: the rows kernel's block sums added in a fixed order
  if (loss_wave) {
    const double sl0 = (blv[0] + blv[1]) + (blv[2] + blv[3]);
    double sl = sl0;
    for (int off = 32; off > 0; off >>= 1) sl += __shfl_down(sl, off, 64);
    if (lane == 0) a.acc[0] += sl;
  }
}

namespace {

template <int W, int P, int D>
hipError_t rows_launch(const FusedRowsArgs& a, hipStream_t s) {
  constexpr int NW = W >= 128 ? 8 : 4;
  fused_rows_kernel<W, P, P, D, NW><<<a.B / R, 64 * NW, 0, s>>>(a);
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

namespace {

__global__ void permute_rows_kernel(const __bf16* X, const float* T, const int* perm, int64_t M, int in_p,
                                    int out_p, __bf16* Xp, float* Tp) {
  const int cx = in_p / 8, ct = out_p / 4;   // 16-byte pieces per row
  const int64_t total = M * (cx + ct);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / (cx + ct);
    const int c = (int)(e % (cx + ct));
    const int64_t src = perm[i];
    if (c < cx)
      *reinterpret_cast<bf16x8*>(Xp + i * in_p + 8 * c) = *reinterpret_cast<const bf16x8*>(X + src * in_p + 8 * c);
    else
      *reinterpret_cast<f32x4*>(Tp + i * out_p + 4 * (c - cx)) =
          *reinterpret_cast<const f32x4*>(T + src * out_p + 4 * (c - cx));
  }
}

}  // namespace

hipError_t launch_permute_rows(const __bf16* X, const float* T, const int* perm, int64_t M, int in_p, int out_p,
                               __bf16* Xp, float* Tp, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (in_p % 8 || out_p % 4) return hipErrorInvalidValue;
  const int64_t total = M * (in_p / 8 + out_p / 4);
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  permute_rows_kernel<<<grid, 256, 0, s>>>(X, T, perm, M, in_p, out_p, Xp, Tp);
  return hipGetLastError();
}

bool fused_weights_supported(int B) { return B == 256 || B == 512 || B == 1024 || B == 2048 || B == 4096; }

hipError_t launch_fused_weights(const FusedWeightsArgs& a, hipStream_t s) {
  constexpr int NWV = 8;
  if (a.nbl > 256) return hipErrorInvalidValue;   // the loss wave reads at most four sums per lane
  const dim3 g(a.tiles), blk(64 * NWV);
  switch (a.B) {
    case 256: fused_weights_kernel<2, NWV><<<g, blk, 0, s>>>(a); break;
    case 512: fused_weights_kernel<4, NWV><<<g, blk, 0, s>>>(a); break;
    case 1024: fused_weights_kernel<8, NWV><<<g, blk, 0, s>>>(a); break;
    case 2048: fused_weights_kernel<16, NWV><<<g, blk, 0, s>>>(a); break;
    case 4096: fused_weights_kernel<32, NWV><<<g, blk, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hjg
