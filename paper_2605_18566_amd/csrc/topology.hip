// Topology markers of the zero-sublevel set {v <= 0} on 2D slices: connected
// components (4-neighbour), encircled components of the complement (holes),
// Euler characteristic chi = n_comp - beta_1, and the event rules between
// consecutive steps (appendix on vacuole nucleation topology).  One block per
// slice: union-find over the cells in LDS (links always point to a smaller
// index and are set by atomic minimum, so concurrent unions keep a forest).
#include <hip/hip_runtime.h>

#include <string>

#include "hjg.h"
#include "internal.h"

namespace {

constexpr int kTT = 1024;
constexpr int kMaxCells = 16384;

int fail(int code, const std::string& msg) { return hjg_internal_fail(code, msg.c_str()); }

__device__ __forceinline__ int find_root(volatile int* parent, int x) {
  int p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

__device__ __forceinline__ void unite(int* parent, int a, int b) {
  while (true) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(&parent[a], b);   // link the larger root below the smaller
    if (old == a) return;
    a = old;                                     // a was linked meanwhile: retry from its new parent
  }
}

__global__ __launch_bounds__(kTT) void topology_kernel(int ny, int nx, const float* v, int* ncomp, int* beta1,
                                                       int* chi) {
  __shared__ int parent[kMaxCells];
  __shared__ unsigned char inside[kMaxCells];
  __shared__ unsigned char edge[kMaxCells];
  __shared__ int cnt[2];
  const int cells = ny * nx;
  const float* vs = v + (int64_t)blockIdx.x * cells;
  const int tid = threadIdx.x;
  for (int i = tid; i < cells; i += kTT) {
    parent[i] = i;
    inside[i] = vs[i] <= 0.f ? 1 : 0;
    edge[i] = 0;
  }
  if (tid < 2) cnt[tid] = 0;
  __syncthreads();
  for (int i = tid; i < cells; i += kTT) {
    const int x = i % nx, y = i / nx;
    if (x + 1 < nx && inside[i] == inside[i + 1]) unite(parent, i, i + 1);
    if (y + 1 < ny && inside[i] == inside[i + nx]) unite(parent, i, i + nx);
  }
  __syncthreads();
  for (int i = tid; i < cells; i += kTT) parent[i] = find_root(parent, i);
  __syncthreads();
  for (int i = tid; i < cells; i += kTT) {
    const int x = i % nx, y = i / nx;
    if (!inside[i] && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1)) edge[parent[i]] = 1;
  }
  __syncthreads();
  for (int i = tid; i < cells; i += kTT) {
    if (parent[i] == i) {
      if (inside[i]) atomicAdd(&cnt[0], 1);
      else if (!edge[i]) atomicAdd(&cnt[1], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    ncomp[blockIdx.x] = cnt[0];
    beta1[blockIdx.x] = cnt[1];
    chi[blockIdx.x] = cnt[0] - cnt[1];
  }
}

}  // namespace

extern "C" {

int hjg_topology(int32_t B, int32_t ny, int32_t nx, const float* v, int32_t* n_comp, int32_t* beta1, int32_t* chi,
                 void* hip_stream) {
  if (B < 0 || ny < 1 || nx < 1) return fail(HJG_EINVAL, "need B >= 0 and a grid of at least 1 x 1");
  if ((int64_t)ny * nx > kMaxCells) return fail(HJG_EUNSUPPORTED, "slices of at most 16,384 cells (128 x 128)");
  if (B == 0) return HJG_OK;
  if (!v || !n_comp || !beta1 || !chi) return fail(HJG_EINVAL, "v, n_comp, beta1 and chi are required");
  topology_kernel<<<(unsigned)B, kTT, 0, (hipStream_t)hip_stream>>>(ny, nx, v, n_comp, beta1, chi);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HJG_EHIP, std::string("topology_kernel: ") + hipGetErrorString(e));
  return HJG_OK;
}

int hjg_topology_events(int32_t T, const int32_t* chi, const int32_t* beta1, const int32_t* n_comp,
                        int32_t* events) {
  if (T < 0) return fail(HJG_EINVAL, "T must be >= 0");
  if (T > 0 && (!chi || !beta1 || !n_comp || !events)) return fail(HJG_EINVAL, "NULL argument");
  for (int t = 0; t < T; ++t) {
    int e = 0;
    if (t > 0) {
      if (chi[t] - chi[t - 1] < 0) e |= HJG_EVENT_VACUOLE;          // integer form of a drop below -0.5
      if (beta1[t] >= 1 && beta1[t - 1] == 0) e |= HJG_EVENT_CORDON;
      if (n_comp[t] > n_comp[t - 1]) e |= HJG_EVENT_FRAGMENTATION;
    }
    events[t] = e;
  }
  return HJG_OK;
}

}  // extern "C"
