// Fused training step of the surrogate network: two launches per step.
//
// The transposed activations and errors that pass from the first kernel to
// the second are stored in blocks of 64 batch columns: element (feature f,
// batch row b) of an array of F features sits at (b / 64) F 64 + 64 f + b % 64,
// so the 32 feature rows x 16 batch columns that one matrix-core step of the
// second kernel reads lie in one 4 KB span.
//
// Rows kernel: each block takes 16 rows of the batch through every layer
// (forward with SiLU, the loss and its output error, the backward error
// through every hidden layer), keeping the activations, pre-activations and
// errors of its rows in LDS and streaming each layer's bfloat16 weights from
// the cache into registers (the next layer's weights are requested while the
// current layer computes).  It writes the transposed bfloat16 activations
// and errors that the weight gradients contract over the batch.
//
// Weights kernel: each block takes one 32 x 32 tile of one layer's weight
// gradient, contracting the batch on the matrix cores (the waves split the
// batch and their sums are added in a fixed order), sums the bias gradients
// on the tiles of the first column, and applies AdamW to the tile's weights
// in place (with the bfloat16 copies refreshed), or stores the gradient.
//
// Every step's arguments are fixed (its rows of the epoch's permuted training
// set, its learning-rate entry), so an epoch of steps records as one graph
// and no kernel waits on a device counter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hjg {

constexpr int kFusedRows = 16;        // batch rows per block of the rows kernel
constexpr int kFusedMaxHidden = 4;    // hidden layers whose pre-activations stay in LDS
constexpr int kFusedMaxPhases = 2 * (kFusedMaxHidden + 1) - 1;

enum FusedPhaseKind { PH_FWD_HIDDEN = 0, PH_FWD_OUT = 1, PH_BWD = 2 };

// One matrix product of the rows kernel: out[16][N] = src[16][K] W^T with W
// row-major [N][K] (Wb of a layer going forward, its transpose WbT going
// backward); the shapes and epilogues are fixed by the kernel's instance.
struct FusedPhase {
  const __bf16* W;
  const float* bias;   // forward phases: [N]
  __bf16* outT;        // transposed bfloat16 output, N features x B (64-column blocks)
};

struct FusedRowsArgs {
  FusedPhase ph[kFusedMaxPhases];
  const __bf16* X;      // network inputs [M][in_p] (normalised, bfloat16)
  const float* T;       // normalised targets [M][out_p]
  int64_t row0;         // batch row r is row row0 + r of X and T
  int B, in_p, out_p, nout;
  const float* lw;      // loss weight per output column [out_p]
  __bf16* X0T;          // transposed inputs, in_p features x B (64-column blocks)
  double* block_loss;   // [B / 16]
};

struct FusedLayer {
  const __bf16* A;      // errors, transposed: fout x B (64-column blocks)
  const __bf16* Bm;     // the layer's inputs, transposed: fin x B (64-column blocks)
  int fin, fout;
  int64_t woff, boff;   // offsets in the flat parameter vectors
  __bf16* Wb;           // [fout][fin]
  __bf16* WbT;          // [fin][fout]
  int tiles_n, first;   // tiles across fin; first tile index of the layer
};

struct FusedWeightsArgs {
  int L, B, tiles;
  FusedLayer layer[17];
  // AdamW (adam != 0) or gradient store
  int adam;
  float* w;
  float* g;             // gradient store (adam == 0)
  float* m;
  float* v;
  const float* sched;   // this step's {learning rate, 1 - b1^t, 1 - b2^t} (adam != 0)
  float b1, b2, eps, wd;
  // loss: block 0 adds sum(block_loss[0..nbl)) to *acc (fixed order)
  const double* block_loss;
  int nbl;
  double* acc;
};

// The rows kernel is instantiated for hidden widths 64, 128 and 256, padded
// input and output widths 32 or 64 (equal) and 2 to 4 hidden layers.
bool fused_rows_supported(int width, int in_p, int out_p, int depth);
hipError_t launch_fused_rows(const FusedRowsArgs& a, int width, int depth, hipStream_t s);
// The weights kernel is instantiated for batches of 256, 512, 1024, 2048 and 4096 rows.
bool fused_weights_supported(int B);
hipError_t launch_fused_weights(const FusedWeightsArgs& a, hipStream_t s);

// Xp[i] = X[perm[i]], Tp[i] = T[perm[i]] for i < M (an epoch's batch order).
hipError_t launch_permute_rows(const __bf16* X, const float* T, const int* perm, int64_t M, int in_p, int out_p,
                               __bf16* Xp, float* Tp, hipStream_t s);

}  // namespace hjg
