// Surrogate-network kernels: bfloat16 matrix-core GEMM with fused epilogues,
// loss, bias gradients, AdamW, data preparation, and the compaction used by
// the surrogate-accelerated sweep's fallback.
#include <algorithm>

#include <cmath>

#include "mlp.h"

namespace hjg {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kTN = 64, kTK = 32;   // block tile columns; K ranges are multiples of kTK
constexpr int kKS = 256;                       // K range staged in LDS per barrier
constexpr int kLdsK = kKS + 8;                 // padded LDS row (528 bytes, 16-byte aligned)

// logistic function with the hardware reciprocal (shared by every network kernel)
__device__ __forceinline__ float sigmoidf_(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Block tile TM x 64 (TM = 64 or 32), waves as (TM/32) x 2 sub-tiles of
// 32 x 32, each sub-tile one v_mfma_f32_32x32x16_bf16 chain (two per 32-deep
// K slice); 4 TM threads.  The 32-row form doubles the blocks of the small
// training shapes, whose single tile per CU cannot hide its load latency.
// Operand lanes: A[i = l%32][k = 8(l/32)..+7], B[k = 8(l/32)..+7][j = l%32];
// accumulator lane l holds rows 8(v/4) + 4(l/32) + v%4 of column l%32.
template <int EPI, int TM>
__global__ __launch_bounds__(4 * TM) void gemm_nt_kernel(GemmArgs g) {
  constexpr int kThr = 4 * TM, BR = kTN / TM;   // threads; B rows per loader thread
  __shared__ __attribute__((aligned(16))) __bf16 As[TM][kLdsK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[kTN][kLdsK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * kTN;
  int kb = 0, ke = g.K;
  if (EPI == EPI_DW) {
    kb = blockIdx.z * g.k_per_split;
    ke = min(g.K, kb + g.k_per_split);
  }
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  // Up to kKS of the K range per round: every load of the round is issued
  // before one barrier (the small training shapes are latency bound), then
  // the MFMA chain runs in ascending k.
  const int lr = tid >> 2, lk = (tid & 3) * 8;   // loader: row (+ TM b for B), k offset (+ 32 j)
  const bool arow = m0 + lr < g.M;
  // EPI_DW with pbias: the first column of blocks also sums its A rows
  // (row lr, k offsets lk + 32 j) for the bias gradient
  const bool rowsum = EPI == EPI_DW && g.pbias && blockIdx.x == 0;
  float bsum = 0.f;
  for (int k0 = kb; k0 < ke; k0 += kKS) {
    const int kc = min(kKS, ke - k0);
    bf16x8 va[kKS / kTK], vb[BR][kKS / kTK];
#pragma unroll
    for (int j = 0; j < kKS / kTK; ++j) {
      if (j * kTK >= kc) break;
      if (arow) va[j] = *reinterpret_cast<const bf16x8*>(g.A + (int64_t)(m0 + lr) * g.lda + k0 + j * kTK + lk);
      else
#pragma unroll
        for (int e = 0; e < 8; ++e) va[j][e] = (__bf16)0.f;
#pragma unroll
      for (int b = 0; b < BR; ++b) {
        const int row = n0 + lr + TM * b;
        if (row < g.N) vb[b][j] = *reinterpret_cast<const bf16x8*>(g.B + (int64_t)row * g.ldb + k0 + j * kTK + lk);
        else
#pragma unroll
          for (int e = 0; e < 8; ++e) vb[b][j][e] = (__bf16)0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < kKS / kTK; ++j) {
      if (j * kTK >= kc) break;
      *reinterpret_cast<bf16x8*>(&As[lr][j * kTK + lk]) = va[j];
#pragma unroll
      for (int b = 0; b < BR; ++b) *reinterpret_cast<bf16x8*>(&Bs[lr + TM * b][j * kTK + lk]) = vb[b][j];
    }
    __syncthreads();
    if (rowsum) {
#pragma unroll
      for (int j = 0; j < kKS / kTK; ++j) {
        if (j * kTK >= kc) break;
        const bf16x8 r = *reinterpret_cast<const bf16x8*>(&As[lr][j * kTK + lk]);
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum += (float)r[e];
      }
    }
#pragma unroll
    for (int ks = 0; ks < kKS; ks += 16) {
      if (ks >= kc) break;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (rowsum) {
    bsum += __shfl_xor(bsum, 1);
    bsum += __shfl_xor(bsum, 2);
    if ((tid & 3) == 0 && arow) g.pbias[(int64_t)blockIdx.z * g.M + m0 + lr] = bsum;
  }
  const int n = n0 + wn * 32 + (lane & 31);
  // transposed bf16 copies go through an LDS tile so their stores are
  // coalesced rows of the transposed output
  __shared__ __attribute__((aligned(16))) __bf16 Ts[kTN][TM + 8];
  const bool transposed = (EPI == EPI_BWD_DX) || (EPI == EPI_FWD_HIDDEN && g.outbT);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int ml = wm * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
    const int m = m0 + ml;
    if (m >= g.M || n >= g.N) continue;
    const float c = acc[v];
    if (EPI == EPI_FWD_HIDDEN) {
      const float z = c + g.bias[n];
      if (g.outf) g.outf[(int64_t)m * g.ldo + n] = z;
      const __bf16 s = (__bf16)(z * sigmoidf_(z));
      if (g.outb) g.outb[(int64_t)m * g.ldob + n] = s;
      if (g.outbT) Ts[n - n0][ml] = s;
    } else if (EPI == EPI_FWD_OUT) {
      g.outf[(int64_t)m * g.ldo + n] = c + g.bias[n];
    } else if (EPI == EPI_BWD_DX) {
      const float z = g.zprev[(int64_t)m * g.ldz + n];
      const float sg = sigmoidf_(z);
      const __bf16 d = (__bf16)(c * sg * (1.0f + z * (1.0f - sg)));
      g.outb[(int64_t)m * g.ldob + n] = d;
      Ts[n - n0][ml] = d;
    } else {
      g.outf[((int64_t)blockIdx.z * g.M + m) * g.ldo + n] = c;
    }
  }
  if (transposed) {
    __syncthreads();
    for (int e = tid; e < kTN * (TM / 8); e += kThr) {
      const int r = e / (TM / 8), c = (e % (TM / 8)) * 8;
      const int nn = n0 + r, mm = m0 + c;
      if (nn >= g.N || mm >= g.M) continue;
      __bf16* dst = g.outbT + (int64_t)nn * g.ldobT + mm;
      if (mm + 8 <= g.M && (((uintptr_t)dst) & 15) == 0) {
        *reinterpret_cast<bf16x8*>(dst) = *reinterpret_cast<const bf16x8*>(&Ts[r][c]);
      } else {
        for (int q = 0; q < 8 && mm + q < g.M; ++q) dst[q] = Ts[r][c + q];
      }
    }
  }
}

__global__ __launch_bounds__(256) void sum_splits_kernel(const float* part, int splits, int M, int N, int ld,
                                                         float* dst, int ldd, const float* pbias, float* bdst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t MN = (int64_t)M * N;
  if (i < MN) {
    const int m = (int)(i / N), n = (int)(i % N);
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[((int64_t)z * M + m) * ld + n];
    dst[(int64_t)m * ldd + n] = s;
  } else if (pbias && i < MN + M) {
    const int m = (int)(i - MN);
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += pbias[(int64_t)z * M + m];
    bdst[m] = s;
  }
}

__global__ __launch_bounds__(256) void mse_kernel(const float* Y, const float* T, const float* w, int B, int cols,
                                                  int ld, __bf16* dY, __bf16* dYT, double* block_loss) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (i < (int64_t)B * ld) {
    const int r = (int)(i / ld), c = (int)(i % ld);
    float d = 0.f;
    if (c < cols) {
      const float diff = Y[i] - T[i];
      l = (double)w[c] * (double)diff * (double)diff;
      d = 2.0f * w[c] * diff / (float)B;
    }
    dY[i] = (__bf16)d;
    dYT[(int64_t)c * B + r] = (__bf16)d;
  }
  __shared__ double red[256];
  red[threadIdx.x] = l;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_loss[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void adamw_kernel(float* w, const float* g, float* m, float* v, int64_t count,
                                                    float lr, float b1, float b2, float eps, float wd, float bc1,
                                                    float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  w[i] = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
}

// AdamW with the step's learning rate and bias corrections formed on the
// device from the step counters ctr = {global step k, optimizer steps done,
// batch of the epoch}: cosine schedule lr_min + (lr - lr_min)(1 + cos(pi k/total))/2.
// The schedule (one cosine and two powers in float64) is formed once per
// block.  With tab, each weight (not bias) also refreshes its bfloat16 copies.
__global__ __launch_bounds__(256) void adamw_sched_kernel(float* w, const float* g, float* m, float* v, int64_t count,
                                                          const int64_t* ctr, double lr_max, double lr_min,
                                                          int64_t total, float b1, float b2, float eps, float wd,
                                                          LayerTab tab) {
  __shared__ float sched[3];
  if (threadIdx.x == 0) {
    const double k = (double)ctr[0], step = (double)(ctr[1] + 1);
    sched[0] = (float)(lr_min + 0.5 * (lr_max - lr_min) * (1.0 + cos(M_PI * k / (double)total)));
    sched[1] = (float)(1.0 - pow((double)b1, step));
    sched[2] = (float)(1.0 - pow((double)b2, step));
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float lr = sched[0], bc1 = sched[1], bc2 = sched[2];
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
  w[i] = wi;
  for (int l = 0; l < tab.L; ++l) {
    const int64_t e = i - tab.woff[l];
    if (e >= 0 && e < (int64_t)tab.fin[l] * tab.fout[l]) {
      const int r = (int)(e / tab.fin[l]), c = (int)(e % tab.fin[l]);
      const __bf16 b = (__bf16)wi;
      tab.Wb[l][e] = b;
      tab.WbT[l][(int64_t)c * tab.fout[l] + r] = b;
    }
  }
}

__global__ void advance_counters_kernel(int64_t* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctr[0] += 1;
    ctr[1] += 1;
    ctr[2] += 1;
  }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* W, int rows, int cols, __bf16* Wb, __bf16* WbT) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  const __bf16 b = (__bf16)W[i];
  Wb[i] = b;
  WbT[(int64_t)c * rows + r] = b;
}

__global__ __launch_bounds__(256) void prep_inputs_kernel(const float* x, int64_t xstride, const float* t, int n,
                                                          int64_t rows, int ld, const float* mean, const float* stdv,
                                                          __bf16* X, __bf16* XT) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * ld) return;
  const int64_t r = i / ld;
  const int c = (int)(i % ld);
  float val = 0.f;
  if (c < n) val = (x[(int64_t)c * xstride + r] - mean[c]) / stdv[c];
  else if (c == n) val = (t[r] - mean[n]) / stdv[n];
  const __bf16 b = (__bf16)val;
  X[i] = b;
  if (XT) XT[(int64_t)c * rows + r] = b;
}

__global__ __launch_bounds__(256) void prep_targets_kernel(const float* v, const float* grad, int n, int64_t rows,
                                                           int ld, const float* mean, const float* stdv, float* T) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * ld) return;
  const int64_t r = i / ld;
  const int c = (int)(i % ld);
  float val = 0.f;
  if (c == 0) val = (v[r] - mean[0]) / stdv[0];
  else if (c <= n) val = (grad[(int64_t)(c - 1) * rows + r] - mean[c]) / stdv[c];
  T[i] = val;
}

__global__ __launch_bounds__(256) void post_outputs_kernel(const float* Y, int n, int64_t rows, int ld,
                                                           const float* mean, const float* stdv, float* v,
                                                           float* grad, int64_t gstride) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  v[r] = Y[r * ld] * stdv[0] + mean[0];
  for (int d = 0; d < n; ++d) grad[(int64_t)d * gstride + r] = Y[r * ld + 1 + d] * stdv[1 + d] + mean[1 + d];
}

__global__ __launch_bounds__(256) void fill_kernel(float* p, float val, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = val;
}

// acc[0] += sum of the block partials (fixed order)
__global__ __launch_bounds__(256) void accumulate_kernel(const double* part, int count, double* acc) {
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += part[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += red[0];
}

__global__ __launch_bounds__(256) void feature_stats_kernel(const float* base, int64_t stride, int64_t rows,
                                                            float* mean, float* stdv) {
  const int f = blockIdx.x;
  const float* src = base + f * stride;
  double s = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    const double x = src[r];
    s += x;
    s2 += x * x;
  }
  __shared__ double a[256], b[256];
  a[threadIdx.x] = s;
  b[threadIdx.x] = s2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) { a[threadIdx.x] += a[threadIdx.x + off]; b[threadIdx.x] += b[threadIdx.x + off]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = a[0] / (double)rows;
    const double var = fmax(b[0] / (double)rows - mu * mu, 0.0);
    const double sd = sqrt(var);
    mean[f] = (float)mu;
    stdv[f] = sd > 1e-6 ? (float)sd : 1.0f;   // a constant feature is left unscaled
  }
}

__global__ __launch_bounds__(256) void gather_kernel(const __bf16* X_all, const float* T_all, const int* perm, int B,
                                                     int ld, int ldt, const int64_t* batch, __bf16* Xb, __bf16* XbT,
                                                     float* Tb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (batch) perm += *batch * B;
  if (i < (int64_t)B * ld) {
    const int r = (int)(i / ld), c = (int)(i % ld);
    const __bf16 x = X_all[(int64_t)perm[r] * ld + c];
    Xb[i] = x;
    XbT[(int64_t)c * B + r] = x;
  }
  if (i < (int64_t)B * ldt) {
    const int r = (int)(i / ldt), c = (int)(i % ldt);
    Tb[i] = T_all[(int64_t)perm[r] * ldt + c];
  }
}

__global__ __launch_bounds__(256) void compact_count_kernel(const uint8_t* flags, int64_t Q, int* block_counts) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int f = (q < Q && flags[q]) ? 1 : 0;
  const int c = __syncthreads_count(f);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = c;
}

// exclusive scan of the block counts in place (one thread; at most a few
// thousand blocks); total written separately
__global__ void compact_scan_kernel(int* counts, int nblocks, int* total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0;
  for (int b = 0; b < nblocks; ++b) {
    const int c = counts[b];
    counts[b] = run;
    run += c;
  }
  *total = run;
}

__global__ __launch_bounds__(256) void compact_write_kernel(const uint8_t* flags, int64_t Q, const int* offsets,
                                                            int* index) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int f = (q < Q && flags[q]) ? 1 : 0;
  __shared__ int pre[256];
  pre[threadIdx.x] = f;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {     // inclusive Hillis-Steele scan
    const int add = (int)threadIdx.x >= off ? pre[threadIdx.x - off] : 0;
    __syncthreads();
    pre[threadIdx.x] += add;
    __syncthreads();
  }
  if (f) index[offsets[blockIdx.x] + pre[threadIdx.x] - 1] = (int)q;
}

__global__ __launch_bounds__(256) void gather_soa_kernel(const float* src, int n, int64_t Q, const int* index,
                                                         int64_t count, float* dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count * n) return;
  const int d = (int)(i / count);
  const int64_t j = i % count;
  dst[(int64_t)d * count + j] = src[(int64_t)d * Q + index[j]];
}

__global__ __launch_bounds__(256) void scatter_soa_kernel(const float* src, int n, int64_t count, const int* index,
                                                          int64_t Q, float* dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count * n) return;
  const int d = (int)(i / count);
  const int64_t j = i % count;
  dst[(int64_t)d * Q + index[j]] = src[(int64_t)d * count + j];
}

unsigned nblk(int64_t work) { return (unsigned)std::max<int64_t>((work + 255) / 256, 1); }

}  // namespace

hipError_t launch_gemm(int epi, const GemmArgs& a, int splits, hipStream_t s) {
  if (a.K % kTK) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)((a.N + kTN - 1) / kTN), gz = (unsigned)(epi == EPI_DW ? splits : 1);
  // 64-row tiles unless they leave compute units without a block (measured:
  // the 32-row form is 5 % faster on 1,024-row batches of a width-128 network,
  // 3 % slower on 4,096-row batches of width 256)
  const bool wide = (int64_t)gx * ((a.M + 63) / 64) * gz >= 256;
  const dim3 grid(gx, (unsigned)((a.M + (wide ? 63 : 31)) / (wide ? 64 : 32)), gz);
#define HJG_GEMM(E)                                                           \
  if (wide) gemm_nt_kernel<E, 64><<<grid, 256, 0, s>>>(a);                    \
  else gemm_nt_kernel<E, 32><<<grid, 128, 0, s>>>(a);                         \
  break;
  switch (epi) {
    case EPI_FWD_HIDDEN: HJG_GEMM(EPI_FWD_HIDDEN)
    case EPI_FWD_OUT: HJG_GEMM(EPI_FWD_OUT)
    case EPI_BWD_DX: HJG_GEMM(EPI_BWD_DX)
    case EPI_DW: HJG_GEMM(EPI_DW)
    default: return hipErrorInvalidValue;
  }
#undef HJG_GEMM
  return hipGetLastError();
}

hipError_t launch_sum_splits(const float* part, int splits, int M, int N, int ld, float* dst, int ldd,
                             const float* pbias, float* bdst, hipStream_t s) {
  if (pbias && !bdst) return hipErrorInvalidValue;
  sum_splits_kernel<<<nblk((int64_t)M * N + (pbias ? M : 0)), 256, 0, s>>>(part, splits, M, N, ld, dst, ldd, pbias,
                                                                           bdst);
  return hipGetLastError();
}

hipError_t launch_mse_loss(const float* Y, const float* T, const float* w, int B, int cols, int ld, __bf16* dY,
                           __bf16* dYT, double* block_loss, int* nblocks, hipStream_t s) {
  const unsigned nb = nblk((int64_t)B * ld);
  *nblocks = (int)nb;
  mse_kernel<<<nb, 256, 0, s>>>(Y, T, w, B, cols, ld, dY, dYT, block_loss);
  return hipGetLastError();
}

hipError_t launch_adamw(float* w, const float* g, float* m, float* v, int64_t count, float lr, float beta1,
                        float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s) {
  adamw_kernel<<<nblk(count), 256, 0, s>>>(w, g, m, v, count, lr, beta1, beta2, eps, wd, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_adamw_sched(float* w, const float* g, float* m, float* v, int64_t count, const int64_t* ctr,
                              double lr_max, double lr_min, int64_t total, float beta1, float beta2, float eps,
                              float wd, const LayerTab* tab, hipStream_t s) {
  LayerTab t{};
  if (tab) {
    if (tab->L < 0 || tab->L > kMaxLayers) return hipErrorInvalidValue;
    t = *tab;
  }
  adamw_sched_kernel<<<nblk(count), 256, 0, s>>>(w, g, m, v, count, ctr, lr_max, lr_min, total, beta1, beta2, eps, wd,
                                                 t);
  return hipGetLastError();
}

hipError_t launch_advance_counters(int64_t* ctr, hipStream_t s) {
  advance_counters_kernel<<<1, 64, 0, s>>>(ctr);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* WbT, hipStream_t s) {
  to_bf16_kernel<<<nblk((int64_t)rows * cols), 256, 0, s>>>(W, rows, cols, Wb, WbT);
  return hipGetLastError();
}

hipError_t launch_prep_inputs(const float* x, int64_t xstride, const float* t, int n, int64_t rows, int ld,
                              const float* mean, const float* stdv, __bf16* X, __bf16* XT, hipStream_t s) {
  prep_inputs_kernel<<<nblk(rows * ld), 256, 0, s>>>(x, xstride, t, n, rows, ld, mean, stdv, X, XT);
  return hipGetLastError();
}

hipError_t launch_prep_targets(const float* v, const float* grad, int n, int64_t rows, int ld, const float* mean,
                               const float* stdv, float* T, hipStream_t s) {
  prep_targets_kernel<<<nblk(rows * ld), 256, 0, s>>>(v, grad, n, rows, ld, mean, stdv, T);
  return hipGetLastError();
}

hipError_t launch_post_outputs(const float* Y, int n, int64_t rows, int ld, const float* mean, const float* stdv,
                               float* v, float* grad, int64_t gstride, hipStream_t s) {
  post_outputs_kernel<<<nblk(rows), 256, 0, s>>>(Y, n, rows, ld, mean, stdv, v, grad, gstride);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, float val, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  fill_kernel<<<nblk(count), 256, 0, s>>>(p, val, count);
  return hipGetLastError();
}

hipError_t launch_accumulate(const double* part, int count, double* acc, hipStream_t s) {
  accumulate_kernel<<<1, 256, 0, s>>>(part, count, acc);
  return hipGetLastError();
}

hipError_t launch_feature_stats(const float* base, int64_t stride, int nf, int64_t rows, float* mean, float* stdv,
                                hipStream_t s) {
  feature_stats_kernel<<<nf, 256, 0, s>>>(base, stride, rows, mean, stdv);
  return hipGetLastError();
}

hipError_t launch_gather(const __bf16* X_all, const float* T_all, const int* perm, int B, int ld, int ldt,
                         const int64_t* batch, __bf16* Xb, __bf16* XbT, float* Tb, hipStream_t s) {
  gather_kernel<<<nblk((int64_t)B * std::max(ld, ldt)), 256, 0, s>>>(X_all, T_all, perm, B, ld, ldt, batch, Xb, XbT,
                                                                      Tb);
  return hipGetLastError();
}

hipError_t launch_compact_count(const uint8_t* flags, int64_t Q, int* block_counts, int* nblocks, hipStream_t s) {
  const unsigned nb = nblk(Q);
  *nblocks = (int)nb;
  compact_count_kernel<<<nb, 256, 0, s>>>(flags, Q, block_counts);
  return hipGetLastError();
}

hipError_t launch_compact_scan(int* block_counts, int nblocks, int* total, hipStream_t s) {
  compact_scan_kernel<<<1, 64, 0, s>>>(block_counts, nblocks, total);
  return hipGetLastError();
}

hipError_t launch_compact_write(const uint8_t* flags, int64_t Q, const int* block_offsets, int* index,
                                hipStream_t s) {
  compact_write_kernel<<<nblk(Q), 256, 0, s>>>(flags, Q, block_offsets, index);
  return hipGetLastError();
}

hipError_t launch_gather_soa(const float* src, int n, int64_t Q, const int* index, int64_t count, float* dst,
                             hipStream_t s) {
  if (count == 0) return hipSuccess;
  gather_soa_kernel<<<nblk(count * n), 256, 0, s>>>(src, n, Q, index, count, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_soa(const float* src, int n, int64_t count, const int* index, int64_t Q, float* dst,
                              hipStream_t s) {
  if (count == 0) return hipSuccess;
  scatter_soa_kernel<<<nblk(count * n), 256, 0, s>>>(src, n, count, index, Q, dst);
  return hipGetLastError();
}

}  // namespace hjg
