// Kernel arguments and launchers of the sweep (host <-> kernel boundary inside
// the library; not part of the public C interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace hjg {

constexpr int kThreads = 256;   // threads per block; one query per thread
constexpr int kBlk = 128;       // samples staged in LDS per round (CRN)

// Partial sums of one (query, sample split), all relative to the split's
// running maximum m of the log2-weights:
//   pm  [s][Q] float    m (log2 units)
//   pS  [s][Q] double   sum 2^(a - m)
//   pS2 [s][Q] double   sum 2^(2(a - m))
//   pG  [s][n][Q] float sum 2^(a - m) z
//   pZ  [s][n][Q] float sum z          (FRESH with control variate only)
struct Partials {
  float* m;
  double* S;
  double* S2;
  float* G;
  float* Z;
};

struct SweepArgs {
  int n;
  int64_t Q;
  int N;
  int ns;          // samples per split
  int splits;
  const float* x;      // [n][Q]
  const float* c;      // [Q]
  const float* theta;  // [n][Q] or nullptr
  float sigma;
  const void* table;   // [n][tstride] float32 or bf16 bits (CRN)
  int64_t tstride;
  const float* zd;     // stacked disc pairs on the matrix cores: [N][zs] float32
                       // copy of each sample's 2m planar coordinates, else nullptr
  DatumP dp;
  uint32_t k0, k1, tag;  // Philox key and tag (FRESH)
  int cv;                // FRESH: also accumulate sum z
  int mfma;              // 1: contractions on the matrix cores (bf16 table, n >= 16)
  Partials part;
  const int* done;       // Picard stop flag or nullptr
};

struct FinalizeArgs {
  int n;
  int64_t Q;
  int N;
  int splits;
  float sigma;
  const float* x;
  const float* c;        // coefficient used by the sweep  [Q]
  const float* theta;    // shift used by the sweep [n][Q] or nullptr
  Partials part;
  int cv;                // subtract zbar
  int fresh;             // zbar per query from part.Z, else from zbar_tab
  const double* zbar_tab;  // [n] mean of the common table
  float* v;
  float* grad;
  float* ess;            // or nullptr
  // Picard bookkeeping (picard != 0)
  int picard;
  float* vprev;          // [Q] in: v^(k), out: v^(k+1)
  float* c_out;          // [Q] or nullptr
  uint8_t* flags;        // [Q] or nullptr
  float tol;
  float vfloor;
  double* blockpart;     // [gridDim.x][3]: sum dv^2, sum vprev^2, number of states
                         // whose v or gradient is not finite
  float* c_next;         // [Q] (may alias c)
  float* th_next;        // [n][Q] (may alias theta) or nullptr
  HamP hp;
  const int* done;
};

struct InitArgs {
  int n;
  int64_t Q;
  int K;
  float sigma;
  const float* x;
  const float* p0;       // warm-start gradient or nullptr
  const float* v0;       // warm-start value or nullptr (then v^(0) = l(x))
  DatumP dp;
  HamP hp;
  int tilt;
  float* vprev;
  float* p;              // [n][Q] gradient iterate (the caller's grad buffer)
  float* c;
  float* th;             // or nullptr
  int* done;
  int* iters;
  int* nonfinite;        // reset to 0 (or nullptr)
  double* resid;         // [K]
};

struct ReduceArgs {
  int nblocks;
  const double* blockpart;
  int k;
  float tol;
  double* resid;
  int* done;
  int* iters;
  int* nonfinite;        // out: states of iteration k with a non-finite v or gradient (or nullptr)
};

// A batched launch: block b serves items[b] = (problem, query block, split)
// with probs[problem]; every problem of one launch shares the kernel
// specialisation of the SweepArgs passed alongside.
struct SweepBatch {
  const SweepArgs* probs;
  const int4* items;
  int count;
  int* counter;   // work-queue head (zero before the launch): a persistent grid
                  // of resident blocks takes items in order; nullptr = one block per item
};

hipError_t launch_sweep(const SweepArgs& a, int fresh, int bf16, hipStream_t s, const SweepBatch* b = nullptr);
// A batched per-query launch: block b serves items[b] = (problem, query block).
template <class Args>
struct ItemBatch {
  const Args* args;
  const int2* items;
  int count;
};

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s, const ItemBatch<FinalizeArgs>* b = nullptr);
hipError_t launch_init(const InitArgs& a, hipStream_t s, const ItemBatch<InitArgs>* b = nullptr);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_reduce_batched(const ReduceArgs* args, const int* plist, int count, int k, hipStream_t s);
hipError_t launch_table(int n, int64_t limit, int64_t tstride, uint32_t k0, uint32_t k1, uint32_t tag, int bf16,
                        void* out, hipStream_t s);
hipError_t launch_zbar(int n, int N, int64_t tstride, int bf16, const void* table, double* zbar, hipStream_t s);
// zd[i][2k + e] = table[3k + e][i] (bf16 -> float32, k < m, e < 2), zero up to zs.
hipError_t launch_pair_coords(int m, int N, int64_t tstride, const void* table_bf16, int zs, float* zd, hipStream_t s);
hipError_t launch_philox_words(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t G,
                               uint32_t* out, hipStream_t s);
hipError_t launch_finite_check(const float* a, int64_t count, int* flag, hipStream_t s);
hipError_t launch_fill_ints(int* a, int64_t count, int value, hipStream_t s);

// Time-marching step with the surrogate network as the datum.  Rows of one
// query chunk are r = (q - q0) N + i for q in [q0, q0 + Qc), i < N.
// Points: X0[r][c] = bf16 of the normalised network input at
//   y = x_q + theta_q + sigma z_i (c < n), the previous time (c = n), 0 (c < ld).
struct TubePointsArgs {
  int n;
  int64_t Q, q0, Qc;
  int N;
  const float* x;       // [n][Q]
  const float* theta;   // [n][Q] or nullptr
  float sigma;
  const void* table;    // common table [n][tstride], float32 or bf16 bits
  int64_t tstride;
  int bf16;
  float t_prev;
  const float* mean;    // input normalisation [n + 1]
  const float* stdv;
  int ld;               // padded input width
  __bf16* X0;           // [Qc N][ld]
  const int* done;      // Picard stop flag
};
// Log-sum-exp of one query per block over its N rows: the datum of row r is
// Y[r][0] * ostd + omean (the network's value output), and the partials
// (split 0) take the same form as those of the pair loops.
struct TubeLseArgs {
  int n;
  int64_t Q, q0, Qc;
  int N;
  const float* c;       // [Q]
  const float* theta;   // [n][Q] or nullptr
  float sigma;
  const void* table;
  int64_t tstride;
  int bf16;
  const float* Y;       // [Qc N][ldy]
  int ldy;
  const float* omean;   // value output de-normalisation (device scalars)
  const float* ostd;
  Partials part;
  const int* done;
};
// Fused form for small networks (hidden width 128, padded input width 32,
// up to three hidden layers, n <= 8): one block per query runs the inputs,
// every layer and the value output on the matrix cores with activations in
// LDS, and folds the values into the partials; no rows touch memory.
constexpr int kTubeMaxDepth = 4;
constexpr int kTubeFusedMaxDepth = 3, kTubeFusedMaxN = 8, kTubeFusedWidth = 128, kTubeFusedInP = 32;
struct TubeFusedArgs {
  int n;
  int64_t Q;
  int N;
  int depth;
  const float* x;       // [n][Q]
  const float* theta;   // [n][Q] or nullptr
  float sigma;
  const void* table;
  int64_t tstride;
  int bf16;
  float t_prev;
  const float* mean;    // input normalisation [n + 1]
  const float* stdv;
  const __bf16* W[kTubeMaxDepth + 1];   // [fout][fin] bfloat16: 128 x 32, 128 x 128 ..., out_p x 128
  const float* b[kTubeMaxDepth + 1];
  const float* omean;
  const float* ostd;
  const float* c;
  Partials part;
  const int* done;
};
hipError_t launch_tube_fused(const TubeFusedArgs& a, hipStream_t s);

constexpr int kTubeMaxSamples = 1 << 21;
constexpr int64_t kTubeRowsPerChunk = int64_t(1) << 21;   // network rows per forward pass
hipError_t launch_tube_points(const TubePointsArgs& a, hipStream_t s);
hipError_t launch_tube_lse(const TubeLseArgs& a, hipStream_t s);

// Item index a block of a persistent batched launch serves next: taken from
// the work queue by one thread and shared through LDS; count or more = done.
// The batched launches' problem records and work items are written by the
// host before the launch and only read while it runs.  Reading them through
// the constant address space lets the compiler use scalar loads for them
// (the item index is uniform), and take a field again from the scalar cache
// where it does not keep it in a register, instead of a vector load and a
// wait inside the pair loop.
__device__ __forceinline__ int4 work_item(const int4* items, int b) {
  return *(const int4*)((const __attribute__((address_space(4))) int4*)items + b);
}

__device__ __forceinline__ const SweepArgs& problem_args(const SweepArgs* probs, int p) {
  return *(const SweepArgs*)((const __attribute__((address_space(4))) SweepArgs*)probs + p);
}

__device__ __forceinline__ int next_item(int* counter, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  const int b = *slot;
  __syncthreads();
  // every lane read the same value: make it a scalar, so that the item's
  // record and its problem's arguments are read through the scalar cache
  return __builtin_amdgcn_readfirstlane(b);
}

// Uniform hash grid over agent positions: cell (x, y, z) covers
// [lo + (x, y, z) h, lo + (x+1, y+1, z+1) h); positions outside are clamped
// into the border cells.
struct GridGeom {
  float lo[3];
  float h, inv_h;
  int g[3];
};
constexpr int64_t kMaxGridCells = int64_t(1) << 26;
// pos [3][M]; cell, rank [M]; start [cells + 1] (becomes the exclusive scan
// of the per-cell counts); bsum [ceil((cells + 1) / 4096)]; sorted [M]
// (x, y, z, agent index bits) in cell order.
hipError_t launch_grid_build(const float* pos, int64_t M, const GridGeom& gg, int* cell, int* rank, int* start,
                             int* bsum, float4* sorted, hipStream_t s);
// k (1..8) nearest other agents: idx [k][M], nbr [k][3][M] (either may be
// null); pos is the agents' positions [3][M] the grid was built from.
hipError_t launch_knn(const float4* sorted, const int* start, const float* pos, int64_t M, const GridGeom& gg, int k,
                      int32_t* idx, float* nbr, hipStream_t s);

// Queries per block of the pair-loop kernels: vector ALU, generic matrix
// core, stacked disc pairs on the matrix cores (one query per lane).
constexpr int kQueriesPerBlockValu = 256;
constexpr int kQueriesPerBlockMfma = 128;
constexpr int kQueriesPerBlockPairs = 512;
// Floats per sample in the pair-coordinate copy: 2m rounded up to 8.
constexpr int pair_coord_stride(int m) { return ((2 * m + 7) / 8) * 8; }

// Smallest register bucket that holds n dimensions.
inline int n_bucket(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 48; }

}  // namespace hjg
