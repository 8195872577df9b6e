// Flock support: a uniform hash grid over agent positions and the k nearest
// other agents of every agent (topological neighbour rule of the flocking
// example), whose positions define each agent's target set (a union of balls).
//
// Build: cell of every agent (clamped into the grid), per-cell counts by
// atomics, exclusive scan of the counts, scatter of (x, y, z, index) into cell
// order.  Search: one thread per agent, agents taken in cell order so a wave
// walks neighbouring cells together; cubic shells of cells r = 0, 1, 2, ...
// are scanned until the k-th best squared distance is below the squared
// distance to the nearest cell not yet scanned (so the result is exact for any
// point distribution), and each row of a shell is one contiguous range of the
// cell-ordered array.  Distances are (dx*dx + dy*dy) + dz*dz in float32 with
// every operation rounded on its own; neighbours are ordered by (squared
// distance, index).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace hjg {
namespace {

constexpr int kScanItems = 16;                         // per thread
constexpr int kScanBlock = kThreads * kScanItems;      // 4096 counts per block

__device__ __forceinline__ int cell_coord(float x, float lo, float inv_h, int g) {
  const float u = fminf(fmaxf((x - lo) * inv_h, 0.f), (float)(g - 1));
  return (int)u;
}

__device__ __forceinline__ float dist2_rounded(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

__global__ __launch_bounds__(kThreads) void zero_ints_kernel(int* a, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) a[i] = 0;
}

__global__ __launch_bounds__(kThreads) void grid_count_kernel(const float* pos, int64_t M, GridGeom gg, int* cell,
                                                              int* rank, int* count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= M) return;
  const int cx = cell_coord(pos[i], gg.lo[0], gg.inv_h, gg.g[0]);
  const int cy = cell_coord(pos[M + i], gg.lo[1], gg.inv_h, gg.g[1]);
  const int cz = cell_coord(pos[2 * M + i], gg.lo[2], gg.inv_h, gg.g[2]);
  const int c = (cz * gg.g[1] + cy) * gg.g[0] + cx;
  cell[i] = c;
  rank[i] = atomicAdd(&count[c], 1);
}

// Exclusive scan of v over the block's T threads (Hillis-Steele in LDS).
template <int T>
__device__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[T - 1];
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

// In place: a[b*4096 .. +4095] -> exclusive scan within the block; bsum[b] = block total.
__global__ __launch_bounds__(kThreads) void scan_blocks_kernel(int* a, int64_t count, int* bsum) {
  __shared__ int sh[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < count ? a[base + k] : 0;
    s += v[k];
  }
  int total;
  int run = block_exclusive_scan<kThreads>(s, sh, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < count) a[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One block of 1024 threads: exclusive scan of the (<= 16384) block totals.
__global__ __launch_bounds__(1024) void scan_totals_kernel(int* bsum, int nb) {
  __shared__ int sh[1024];
  const int base = threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < nb ? bsum[base + k] : 0;
    s += v[k];
  }
  int total;
  int run = block_exclusive_scan<1024>(s, sh, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < nb) bsum[base + k] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(kThreads) void scan_add_kernel(int* a, int64_t count, const int* bsum) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) a[i] += bsum[i / kScanBlock];
}

__global__ __launch_bounds__(kThreads) void grid_scatter_kernel(const float* pos, int64_t M, const int* cell,
                                                                const int* rank, const int* start, float4* sorted) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= M) return;
  sorted[start[cell[i]] + rank[i]] = make_float4(pos[i], pos[M + i], pos[2 * M + i], __int_as_float((int)i));
}

// The k nearest so far, ascending in the strict order (distance, index),
// each kept as one 64-bit key: the squared distance's bits (a non-negative
// float orders like its bit pattern) above the agent index, so the order is
// one unsigned comparison.  Positions are read once at the end.
__device__ __forceinline__ uint64_t knn_key(float d2, int j) {
  return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)j;
}

constexpr uint64_t kNoKey = ((uint64_t)0x7F800000u << 32) | 0x7FFFFFFFu;   // (INFINITY, 0x7FFFFFFF)

template <int K>
struct Best {
  uint64_t key[K];

  __device__ void init() {
#pragma unroll
    for (int s = 0; s < K; ++s) key[s] = kNoKey;
  }
  __device__ float d(int s) const { return __uint_as_float((uint32_t)(key[s] >> 32)); }
  __device__ int i(int s) const { return (int)(uint32_t)key[s]; }
  // insert a key without a branch: every comparison with the kept keys is
  // independent, and entry s takes its left neighbour, the new key or itself
  // (a key that is not below the last changes nothing; kNoKey stands for no
  // candidate)
  __device__ void offer(uint64_t k) {
    bool lt[K];
#pragma unroll
    for (int s = 0; s < K; ++s) lt[s] = k < key[s];
#pragma unroll
    for (int s = K - 1; s > 0; --s) key[s] = lt[s - 1] ? key[s - 1] : (lt[s] ? k : key[s]);
    key[0] = lt[0] ? k : key[0];
  }
};

// Candidates s in [a, e): four points requested together, then offered in
// index order (the kept set does not depend on the order of the offers).
template <int K>
__device__ __forceinline__ void scan_range(Best<K>& b, const float4* sorted, int a, int e, int me, float x, float y,
                                           float z) {
  for (int s = a; s < e; s += 4) {
    float4 q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = sorted[min(s + u, e - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = __float_as_int(q[u].w);
      const bool ok = s + u < e && j != me;
      b.offer(ok ? knn_key(dist2_rounded(q[u].x - x, q[u].y - y, q[u].z - z), j) : kNoKey);
    }
  }
}

template <int K>
__global__ __launch_bounds__(kThreads) void knn_kernel(const float4* sorted, const int* start, const float* pos,
                                                       int64_t M, GridGeom gg, int32_t* idx, float* nbr) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= M) return;
  const float4 self = sorted[t];
  const int me = __float_as_int(self.w);
  const float xs[3] = {self.x, self.y, self.z};
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = cell_coord(xs[d], gg.lo[d], gg.inv_h, gg.g[d]);
  Best<K> b;
  b.init();
  // true once every point outside the cells within r (Chebyshev distance in
  // cells) is farther than the k-th distance kept
  auto done = [&](int r) {
    float gap = INFINITY;
    bool covered = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float slack = 1e-5f * (fabsf(gg.lo[d]) + (float)gg.g[d] * gg.h + fabsf(xs[d]));
      if (c[d] - r > 0) {
        covered = false;
        gap = fminf(gap, xs[d] - (gg.lo[d] + (float)(c[d] - r) * gg.h) - slack);
      }
      if (c[d] + r < gg.g[d] - 1) {
        covered = false;
        gap = fminf(gap, gg.lo[d] + (float)(c[d] + r + 1) * gg.h - xs[d] - slack);
      }
    }
    return covered || (gap > 0.f && b.d(K - 1) < gap * gap);
  };
  // cells within 1: the 3 x 3 rows of the block, each one contiguous range of
  // the cell-ordered points; all 18 range bounds are requested together
  {
    int ra[9], re[9];
    const int x0 = max(c[0] - 1, 0), x1 = min(c[0] + 1, gg.g[0] - 1);
#pragma unroll
    for (int w = 0; w < 9; ++w) {
      const int z = c[2] + w / 3 - 1, y = c[1] + w % 3 - 1;
      const bool in = z >= 0 && z < gg.g[2] && y >= 0 && y < gg.g[1];
      const int row = in ? (z * gg.g[1] + y) * gg.g[0] : 0;
      ra[w] = in ? start[row + x0] : 0;
      re[w] = in ? start[row + x1 + 1] : 0;
    }
#pragma unroll
    for (int w = 0; w < 9; ++w) scan_range<K>(b, sorted, ra[w], re[w], me, xs[0], xs[1], xs[2]);
  }
  for (int r = 2; !done(r - 1); ++r) {
    const int z0 = max(c[2] - r, 0), z1 = min(c[2] + r, gg.g[2] - 1);
    const int y0 = max(c[1] - r, 0), y1 = min(c[1] + r, gg.g[1] - 1);
    const int x0 = max(c[0] - r, 0), x1 = min(c[0] + r, gg.g[0] - 1);
    for (int z = z0; z <= z1; ++z) {
      for (int y = y0; y <= y1; ++y) {
        const int row = (z * gg.g[1] + y) * gg.g[0];
        if (abs(z - c[2]) == r || abs(y - c[1]) == r) {
          scan_range<K>(b, sorted, start[row + x0], start[row + x1 + 1], me, xs[0], xs[1], xs[2]);
        } else {
          if (c[0] - r >= 0) scan_range<K>(b, sorted, start[row + c[0] - r], start[row + c[0] - r + 1], me, xs[0], xs[1], xs[2]);
          if (c[0] + r <= gg.g[0] - 1)
            scan_range<K>(b, sorted, start[row + c[0] + r], start[row + c[0] + r + 1], me, xs[0], xs[1], xs[2]);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int j = b.i(s);
    if (idx) idx[(int64_t)s * M + me] = j;
    if (nbr) {
      // an empty slot (fewer than k other agents) keeps the origin
      const bool real = j != 0x7FFFFFFF;
#pragma unroll
      for (int e = 0; e < 3; ++e) nbr[(int64_t)(3 * s + e) * M + me] = real ? pos[(int64_t)e * M + j] : 0.f;
    }
  }
}

}  // namespace

hipError_t launch_grid_build(const float* pos, int64_t M, const GridGeom& gg, int* cell, int* rank, int* start,
                             int* bsum, float4* sorted, hipStream_t s) {
  const int64_t cells = (int64_t)gg.g[0] * gg.g[1] * gg.g[2];
  const int64_t nc = cells + 1;
  const int gm = (int)((M + kThreads - 1) / kThreads);
  const int gc = (int)((nc + kThreads - 1) / kThreads);
  const int nb = (int)((nc + kScanBlock - 1) / kScanBlock);
  zero_ints_kernel<<<gc, kThreads, 0, s>>>(start, nc);
  grid_count_kernel<<<gm, kThreads, 0, s>>>(pos, M, gg, cell, rank, start);
  scan_blocks_kernel<<<nb, kThreads, 0, s>>>(start, nc, bsum);
  scan_totals_kernel<<<1, 1024, 0, s>>>(bsum, nb);
  scan_add_kernel<<<gc, kThreads, 0, s>>>(start, nc, bsum);
  grid_scatter_kernel<<<gm, kThreads, 0, s>>>(pos, M, cell, rank, start, sorted);
  return hipGetLastError();
}

hipError_t launch_knn(const float4* sorted, const int* start, const float* pos, int64_t M, const GridGeom& gg, int k,
                      int32_t* idx, float* nbr, hipStream_t s) {
  const int gm = (int)((M + kThreads - 1) / kThreads);
  switch (k) {
    case 1: knn_kernel<1><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 2: knn_kernel<2><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 3: knn_kernel<3><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 4: knn_kernel<4><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 5: knn_kernel<5><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 6: knn_kernel<6><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    case 7: knn_kernel<7><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
    default: knn_kernel<8><<<gm, kThreads, 0, s>>>(sorted, start, pos, M, gg, idx, nbr); break;
  }
  return hipGetLastError();
}

}  // namespace hjg
