// Topology markers of the zero-sublevel set {v <= 0} on 2D slices: connected
// components (4-neighbour), encircled components of the complement (holes),
// Euler characteristic chi = n_comp - beta_1, and the event rules between
// consecutive steps (appendix on vacuole nucleation topology).  One block per
// slice: union-find over the cells in LDS (links always point to a smaller
// index and are set by atomic minimum, so concurrent unions keep a forest).
#include <hip/hip_runtime.h>

#include <cmath>
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

// Marching squares: one thread per cell.  Corners c0 = (x, y), c1 = (x+1, y),
// c2 = (x+1, y+1), c3 = (x, y+1); edges e0 = c0-c1, e1 = c1-c2, e2 = c2-c3,
// e3 = c3-c0; a corner is inside when v <= level; a crossed edge is cut at
// the linear interpolation point; the saddle cells are decided by the mean of
// the four corners.  Segments are appended through a global counter.
__device__ __forceinline__ float2 edge_point(int e, const float* c, float level, int x, int y) {
  const int a = e, b = (e + 1) & 3;
  const float cx[4] = {0.f, 1.f, 1.f, 0.f}, cy[4] = {0.f, 0.f, 1.f, 1.f};
  const float t = fminf(fmaxf((level - c[a]) / (c[b] - c[a]), 0.f), 1.f);
  return make_float2((float)x + cx[a] + t * (cx[b] - cx[a]), (float)y + cy[a] + t * (cy[b] - cy[a]));
}

__global__ __launch_bounds__(256) void isocontour_kernel(int64_t total, int ny, int nx, const float* v, float level,
                                                         float* seg, int* seg_slice, int64_t max_seg,
                                                         unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t cells = (int64_t)(ny - 1) * (nx - 1);
  const int b = (int)(i / cells);
  const int64_t cc = i % cells;
  const int y = (int)(cc / (nx - 1)), x = (int)(cc % (nx - 1));
  const float* vs = v + (int64_t)b * ny * nx;
  const float c[4] = {vs[(int64_t)y * nx + x], vs[(int64_t)y * nx + x + 1], vs[(int64_t)(y + 1) * nx + x + 1],
                      vs[(int64_t)(y + 1) * nx + x]};
  int in = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) in |= (c[k] <= level ? 1 : 0) << k;
  if (in == 0 || in == 15) return;
  int pa[2], pb[2], np = 0;
  if (in == 5 || in == 10) {
    const bool centre_in = 0.25f * (c[0] + c[1] + c[2] + c[3]) <= level;
    // cut off the outside corners if the centre is inside, else the inside ones;
    // the edges meeting at corner k are e(k-1) and e(k)
    for (int k = 0; k < 4; ++k) {
      const bool corner_in = (in >> k) & 1;
      if (corner_in != centre_in) {
        pa[np] = (k + 3) & 3;
        pb[np] = k;
        ++np;
      }
    }
  } else {
    int e0 = -1;
    for (int e = 0; e < 4; ++e) {
      if (((in >> e) & 1) != ((in >> ((e + 1) & 3)) & 1)) {
        if (e0 < 0) e0 = e;
        else {
          pa[0] = e0;
          pb[0] = e;
          np = 1;
        }
      }
    }
  }
  for (int k = 0; k < np; ++k) {
    const float2 p = edge_point(pa[k], c, level, x, y), q = edge_point(pb[k], c, level, x, y);
    const unsigned long long slot = atomicAdd(count, 1ull);
    if ((int64_t)slot < max_seg) {
      *reinterpret_cast<float4*>(seg + 4 * slot) = make_float4(p.x, p.y, q.x, q.y);
      if (seg_slice) seg_slice[slot] = b;
    }
  }
}

// Separable Gaussian smoothing of one slice per block in LDS: rows, then
// columns, with mirror extension about the outer cell edges
// (d c b a | a b c d | d c b a).
constexpr int kMaxTaps = 65;
struct SmoothTaps {
  int radius;
  float w[kMaxTaps];
};

__device__ __forceinline__ int mirror(int i, int n) {
  while (i < 0 || i >= n) i = i < 0 ? -i - 1 : 2 * n - i - 1;
  return i;
}

__global__ __launch_bounds__(kTT) void smooth_kernel(int ny, int nx, const float* v, SmoothTaps T, float* out) {
  __shared__ float a[kMaxCells];
  __shared__ float b[kMaxCells];
  const int cells = ny * nx;
  const float* vs = v + (int64_t)blockIdx.x * cells;
  float* os = out + (int64_t)blockIdx.x * cells;
  for (int i = threadIdx.x; i < cells; i += kTT) a[i] = vs[i];
  __syncthreads();
  for (int i = threadIdx.x; i < cells; i += kTT) {
    const int x = i % nx, y = i / nx;
    float acc = 0.f;
    for (int k = -T.radius; k <= T.radius; ++k) acc = fmaf(T.w[k + T.radius], a[y * nx + mirror(x + k, nx)], acc);
    b[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cells; i += kTT) {
    const int x = i % nx, y = i / nx;
    float acc = 0.f;
    for (int k = -T.radius; k <= T.radius; ++k) acc = fmaf(T.w[k + T.radius], b[mirror(y + k, ny) * nx + x], acc);
    os[i] = acc;
  }
}

__global__ void zero_count_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

}  // namespace

extern "C" {

int hjg_isocontour(int32_t B, int32_t ny, int32_t nx, const float* v, float level, float* seg, int32_t* seg_slice,
                   int64_t max_seg, int64_t* count, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_isocontour");
  if (B < 0 || ny < 1 || nx < 1 || max_seg < 0) return fail(HJG_EINVAL, "need B >= 0, a grid of at least 1 x 1, max_seg >= 0");
  if ((int64_t)B * ny * nx > ((int64_t)1 << 40)) return fail(HJG_EINVAL, "too many grid values");
  if (!count) return fail(HJG_EINVAL, "count is required");
  if (max_seg > 0 && !seg) return fail(HJG_EINVAL, "seg is required when max_seg > 0");
  if (B > 0 && !v) return fail(HJG_EINVAL, "v is required");
  hipStream_t st = (hipStream_t)hip_stream;
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(count);
  zero_count_kernel<<<1, 64, 0, st>>>(cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HJG_EHIP, std::string("isocontour: ") + hipGetErrorString(e));
  const int64_t total = (int64_t)B * (ny - 1) * (nx - 1);
  if (total > 0) {
    isocontour_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(total, ny, nx, v, level, seg, seg_slice,
                                                                       max_seg, cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(HJG_EHIP, std::string("isocontour: ") + hipGetErrorString(e));
  }
  return HJG_OK;
}


int hjg_topology(int32_t B, int32_t ny, int32_t nx, const float* v, int32_t* n_comp, int32_t* beta1, int32_t* chi,
                 void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_topology");
  if (B < 0 || ny < 1 || nx < 1) return fail(HJG_EINVAL, "need B >= 0 and a grid of at least 1 x 1");
  if ((int64_t)ny * nx > kMaxCells) return fail(HJG_EUNSUPPORTED, "slices of at most 16,384 cells (128 x 128)");
  if (B == 0) return HJG_OK;
  if (!v || !n_comp || !beta1 || !chi) return fail(HJG_EINVAL, "v, n_comp, beta1 and chi are required");
  topology_kernel<<<(unsigned)B, kTT, 0, (hipStream_t)hip_stream>>>(ny, nx, v, n_comp, beta1, chi);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HJG_EHIP, std::string("topology_kernel: ") + hipGetErrorString(e));
  return HJG_OK;
}

int hjg_smooth_slices(int32_t B, int32_t ny, int32_t nx, const float* v, double sigma, float* out,
                      void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_smooth_slices");
  if (B < 0 || ny < 1 || nx < 1) return fail(HJG_EINVAL, "need B >= 0 and a grid of at least 1 x 1");
  if ((int64_t)ny * nx > kMaxCells) return fail(HJG_EUNSUPPORTED, "slices of at most 16,384 cells (128 x 128)");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(HJG_EINVAL, "sigma must be finite and > 0");
  SmoothTaps T{};
  T.radius = (int)(4.0 * sigma + 0.5);               // four standard deviations
  if (2 * T.radius + 1 > kMaxTaps) return fail(HJG_EUNSUPPORTED, "sigma at most 8 cells");
  if (B == 0) return HJG_OK;
  if (!v || !out) return fail(HJG_EINVAL, "v and out are required");
  double wsum = 0.0, w[kMaxTaps];
  for (int k = -T.radius; k <= T.radius; ++k) wsum += (w[k + T.radius] = std::exp(-0.5 * k * k / (sigma * sigma)));
  for (int k = 0; k <= 2 * T.radius; ++k) T.w[k] = (float)(w[k] / wsum);
  smooth_kernel<<<(unsigned)B, kTT, 0, (hipStream_t)hip_stream>>>(ny, nx, v, T, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HJG_EHIP, std::string("smooth_kernel: ") + hipGetErrorString(e));
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
