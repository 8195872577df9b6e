// Fused training step of the surrogate network: two launches per step.
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
// gradient, contracting the batch on the matrix cores (the four waves split
// the batch and their sums are added in a fixed order), sums the bias
// gradients on the tiles of the first column, and applies AdamW to the tile's
// weights in place (with the bfloat16 copies refreshed), or stores the
// gradient.  The last block to finish advances the step counters.
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
  __bf16* outT;        // transposed bfloat16 output [N][B]
};

struct FusedRowsArgs {
  FusedPhase ph[kFusedMaxPhases];
  const __bf16* X;      // network inputs [M][in_p] (normalised, bfloat16)
  const float* T;       // normalised targets [M][out_p]
  const int* perm;      // batch row r is row perm[batch B + r] of X and T, or nullptr (row r)
  const int64_t* batch; // device batch index within the epoch, or nullptr (0)
  int B, in_p, out_p, nout;
  const float* lw;      // loss weight per output column [out_p]
  __bf16* X0T;          // transposed inputs [in_p][B]
  double* block_loss;   // [B / 16]
};

struct FusedLayer {
  const __bf16* A;      // errors, transposed: [fout][B]
  const __bf16* Bm;     // the layer's inputs, transposed: [fin][B]
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
  const int64_t* ctr;   // {global step, optimizer steps done, batch of the epoch}, advanced by the last block
  int* ticket;          // zero between steps
  double lr_max, lr_min;
  int64_t total;
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
hipError_t launch_fused_weights(const FusedWeightsArgs& a, hipStream_t s);

}  // namespace hjg
