// Kernels of the surrogate network and of the surrogate-accelerated sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hjg {

// C[m][n] = sum_k A[m][k] B[n][k] with bfloat16 operands (both k-contiguous),
// float32 accumulation on the matrix cores, K a multiple of 32, and one of
// these epilogues.
enum GemmEpi {
  EPI_FWD_HIDDEN = 0,  // z = C + bias: outf = z (float32), outb/outbT = silu(z) (bfloat16, and transposed)
  EPI_FWD_OUT = 1,     // outf = C + bias
  EPI_BWD_DX = 2,      // dz = C * silu'(zprev): outb/outbT = dz (bfloat16)
  EPI_DW = 3           // split-K partial: outf[z][m][n] = C over the split's K range
};

struct GemmArgs {
  const __bf16* A;
  int lda;
  const __bf16* B;
  int ldb;
  int M, N, K;
  int k_per_split;     // EPI_DW: blockIdx.z covers [z kps, (z+1) kps)
  const float* bias;   // [N]
  float* outf;
  int ldo;
  __bf16* outb;        // [M][ldob] or nullptr
  int ldob;
  __bf16* outbT;       // [N][ldobT] or nullptr
  int ldobT;
  const float* zprev;  // EPI_BWD_DX: [M][ldz]
  int ldz;
  float* pbias;        // EPI_DW: row sums of A over each split's K range, [splits][M], or nullptr
};

hipError_t launch_gemm(int epi, const GemmArgs& a, int splits, hipStream_t s);
// dst[m][n] = sum_z part[z][m][n] for m < M, n < N (row stride ld); with pbias
// also bdst[m] = sum_z pbias[z][m]
hipError_t launch_sum_splits(const float* part, int splits, int M, int N, int ld, float* dst, int ldd,
                             const float* pbias, float* bdst, hipStream_t s);
// dY = 2 w_j (Y - T) / B (bfloat16 and transposed); loss partial sums per block (float64)
hipError_t launch_mse_loss(const float* Y, const float* T, const float* w, int B, int cols, int ld, __bf16* dY,
                           __bf16* dYT, double* block_loss, int* nblocks, hipStream_t s);
// AdamW whose learning rate and bias corrections come from device step
// counters ctr = {global step, optimizer steps done, batch of the epoch}.
// With a layer table, every updated weight is also written to its layer's
// bfloat16 copies (plain [fout][fin] and transposed).
constexpr int kMaxLayers = 17;
struct LayerTab {
  int L;
  int64_t woff[kMaxLayers];   // first weight of layer l in the flat parameter vector
  int fin[kMaxLayers], fout[kMaxLayers];
  __bf16* Wb[kMaxLayers];
  __bf16* WbT[kMaxLayers];
};
hipError_t launch_adamw_sched(float* w, const float* g, float* m, float* v, int64_t count, const int64_t* ctr,
                              double lr_max, double lr_min, int64_t total, float beta1, float beta2, float eps,
                              float wd, const LayerTab* tab, hipStream_t s);
// ctr[0..2] += 1 (one thread)
hipError_t launch_advance_counters(int64_t* ctr, hipStream_t s);
hipError_t launch_adamw(float* w, const float* g, float* m, float* v, int64_t count, float lr, float beta1,
                        float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s);
// bfloat16 copies of a float32 [rows][cols] matrix, plain and transposed
hipError_t launch_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* WbT, hipStream_t s);
// network inputs: X[r][c] = (xt_c(r) - mean_c) / std_c for c < nin, 0 for c < ld (bfloat16, and transposed)
// (x [n] rows with row stride xstride, t [rows]); XT may be nullptr
hipError_t launch_prep_inputs(const float* x, int64_t xstride, const float* t, int n, int64_t rows, int ld,
                              const float* mean, const float* stdv, __bf16* X, __bf16* XT, hipStream_t s);
// targets: T[r][0] = (v - mean_0)/std_0, T[r][1+d] = (grad[d] - mean_{1+d})/std_{1+d}
hipError_t launch_prep_targets(const float* v, const float* grad, int n, int64_t rows, int ld, const float* mean,
                               const float* stdv, float* T, hipStream_t s);
// network outputs back to (v, grad [n][rows])
hipError_t launch_post_outputs(const float* Y, int n, int64_t rows, int ld, const float* mean, const float* stdv,
                               float* v, float* grad, int64_t gstride, hipStream_t s);
hipError_t launch_fill(float* p, float val, int64_t count, hipStream_t s);
hipError_t launch_accumulate(const double* part, int count, double* acc, hipStream_t s);
// mean and std (float64 sums) of each of `nf` features: feature f of row r is
// src_f[r] with src_f = base + f * stride
hipError_t launch_feature_stats(const float* base, int64_t stride, int nf, int64_t rows, float* mean, float* stdv,
                                hipStream_t s);
// batch gather: rows perm[r] of X_all [M][ld] and T_all [M][ldt]
// rows perm[batch * B + r] (batch from device memory, or 0 when null)
hipError_t launch_gather(const __bf16* X_all, const float* T_all, const int* perm, int B, int ld, int ldt,
                         const int64_t* batch, __bf16* Xb, __bf16* XbT, float* Tb, hipStream_t s);
// deterministic stream compaction of the states with flag != 0
hipError_t launch_compact_count(const uint8_t* flags, int64_t Q, int* block_counts, int* nblocks, hipStream_t s);
hipError_t launch_compact_scan(int* block_counts, int nblocks, int* total, hipStream_t s);
hipError_t launch_compact_write(const uint8_t* flags, int64_t Q, const int* block_offsets, int* index,
                                hipStream_t s);
// gather / scatter of SoA state arrays by an index list
hipError_t launch_gather_soa(const float* src, int n, int64_t Q, const int* index, int64_t count, float* dst,
                             hipStream_t s);
hipError_t launch_scatter_soa(const float* src, int n, int64_t count, const int* index, int64_t Q, float* dst,
                              hipStream_t s);

}  // namespace hjg
