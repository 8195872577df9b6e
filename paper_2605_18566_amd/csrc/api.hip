// Host runtime and C interface: context, workspace, argument checks,
// common-table cache, launch planning and the graph-recorded Picard loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdlib>
#include <cstring>
#include <string>
#include <fstream>
#include <sstream>
#include <vector>

#include "hjg.h"
#include "internal.h"
#include "kernels.h"

using namespace hjg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HJG_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(HJG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

// Scratch of hjg_value_grad_noalloc: one fixed array per GPU (the code
// object's copy on each device), never allocated or freed by the library.
// Host code uses only the per-device address taken from hipGetSymbolAddress.
namespace {
constexpr size_t kNoallocScratchBytes = size_t(HJG_NOALLOC_SCRATCH_MIB) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

struct hjg_ctx {
  int device = 0;
  void* scratch = nullptr;     // this device's address of the no-allocation scratch
  hipStream_t cap = nullptr;   // stream used only to record graphs
  // side streams and events of a batched recording: the pair loops of one
  // Picard level become parallel graph branches
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kSide] = {};
  // workspace
  DevBuf pm, pS, pS2, pG, pZ, vprev, cwork, thwork, blockpart, resid, ctrl, table, zbar;
  DevBuf g_cell, g_rank, g_start, g_bsum, g_sorted;   // hash grid of the flock search
  // common-table cache
  bool table_valid = false;
  uint64_t t_seed = 0;
  uint32_t t_pid = 0, t_step = 0;
  int t_n = 0, t_N = 0, t_bf16 = 0;
  int64_t t_stride = 0;
  int t_zd = 0;          // the table buffer also holds the pair-coordinate copy
  int64_t t_zoff = 0;    // its byte offset
  int zbar_valid = 0;
  // recorded Picard graphs
  struct Graph {
    std::vector<char> key;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  // optional timing of the pair-loop kernels: HIP events around each sweep
  int timing = 0;
  std::vector<hipEvent_t> ev;   // [2 * kMaxTimed]: begin/end per sweep launch
  int last_pairs = 0;           // event pairs used by the last call
  // tuning table: sample-split targets chosen by the autotuner
  std::map<std::string, int> tuning;
  // the last batched plan (workspace, argument records, work items, graph)
  struct BatchPlan {
    std::vector<char> key;
    DevBuf ws, args, items;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t replay_ev = nullptr;             // recorded after each replay
    std::vector<int64_t> resid_off, ctrl_off;   // per problem, bytes into ws
    std::vector<int> K;
  } batch;
};

namespace {
constexpr int kMaxTimed = 256;
// Device control words of a context (ctx->ctrl): 0 Picard stop flag, 1
// executed iterations, 2 finiteness flag of hjg_value_grad, 3 that of the
// flock search, 4 Picard count of states with a non-finite output.
constexpr int kCtrlWords = 8;
constexpr int kCtrlNonfinite = 4;
}

namespace {

void drop_batch_graph(hjg_ctx* ctx) {
  if (ctx->batch.exec) (void)hipGraphExecDestroy(ctx->batch.exec);
  if (ctx->batch.graph) (void)hipGraphDestroy(ctx->batch.graph);
  ctx->batch.exec = nullptr;
  ctx->batch.graph = nullptr;
  ctx->batch.key.clear();
}

void drop_graphs(hjg_ctx* ctx) {
  for (auto& g : ctx->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  ctx->graphs.clear();
  drop_batch_graph(ctx);
}

// Grow a workspace buffer; any growth invalidates recorded graphs (they hold
// raw addresses) and waits for the device first so no kernel still uses it.
int ensure(hjg_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes) return HJG_OK;
  HJG_HIP(hipDeviceSynchronize());
  drop_graphs(ctx);
  if (b.p) HJG_HIP(hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = std::max<size_t>(bytes, 256);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(HJG_ENOMEM, "device workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  b.bytes = want;
  if (&b == &ctx->table) ctx->table_valid = false;
  return HJG_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

int check_datum(const hjg_problem* p);

int check_problem(const hjg_problem* p) {
  if (!p) return fail(HJG_EINVAL, "problem is NULL");
  if (p->n < 1 || p->n > kMaxN) return fail(HJG_EINVAL, "n must be in [1, 48]");
  if (!finite_pos(p->nu)) return fail(HJG_EINVAL, "nu must be finite and > 0");
  if (!(std::isfinite(p->eta) && p->eta >= 0)) return fail(HJG_EINVAL, "eta must be finite and >= 0");
  if (!finite_pos(p->c_min) || !finite_pos(p->c_max) || p->c_min > p->c_max)
    return fail(HJG_EINVAL, "need 0 < c_min <= c_max, both finite");
  if (p->problem_id >= (1u << 16)) return fail(HJG_EINVAL, "problem_id must be < 65536");
  if (p->sample_mode != HJG_S_FRESH && p->sample_mode != HJG_S_CRN_STEP)
    return fail(HJG_EINVAL, "unknown sample_mode");
  if (p->sample_mode == HJG_S_FRESH && p->n > 16)
    return fail(HJG_EUNSUPPORTED, "fresh draws are supported for n <= 16; use a common table");
  switch (p->ham) {
    case HJG_H_QUADRATIC:
    case HJG_H_ZERO:
      break;
    case HJG_H_DUBINS_PAIRS:
      if (p->n % 3) return fail(HJG_EINVAL, "Dubins pairs need n = 3m");
      for (int i = 0; i < 4; ++i)
        if (!std::isfinite(p->ham_p[i])) return fail(HJG_EINVAL, "ham_p must be finite");
      break;
    case HJG_H_PURSUIT_EVASION:
      if (p->n % 3 || p->n < 6 || p->n > 48) return fail(HJG_EINVAL, "the pursuit game needs n = 3m, 2 <= m <= 16");
      for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->ham_p[i])) return fail(HJG_EINVAL, "ham_p must be finite");
      if (!(p->ham_p[2] >= 0)) return fail(HJG_EINVAL, "u_max must be >= 0");
      break;
    case HJG_H_MURMURATION:
      if (p->n != 4) return fail(HJG_EINVAL, "the murmuration Hamiltonian needs n = 4");
      for (int i = 0; i < 6; ++i)
        if (!std::isfinite(p->ham_p[i])) return fail(HJG_EINVAL, "ham_p must be finite");
      break;
    case HJG_H_ROCKETS:
      if (p->n != 3) return fail(HJG_EINVAL, "the rockets game needs n = 3");
      for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->ham_p[i])) return fail(HJG_EINVAL, "ham_p must be finite");
      if (!(p->ham_p[2] >= 0)) return fail(HJG_EINVAL, "u_max must be >= 0");
      break;
    case HJG_H_DOUBLE_INTEGRATOR:
      if (p->n != 2 && p->n != 4 && p->n != 6) return fail(HJG_EINVAL, "the double integrator needs n = 2, 4 or 6");
      if (!(std::isfinite(p->ham_p[0]) && p->ham_p[0] >= 0)) return fail(HJG_EINVAL, "u_max must be >= 0");
      if (!std::isfinite(p->ham_p[1])) return fail(HJG_EINVAL, "ham_p must be finite");
      break;
    default:
      return fail(HJG_EINVAL, "unknown Hamiltonian");
  }
  return check_datum(p);
}

// The state dimension and the datum fields (kind, parameters, auxiliary data).
int check_datum(const hjg_problem* p) {
  if (!p) return fail(HJG_EINVAL, "problem is NULL");
  if (p->n < 1 || p->n > kMaxN) return fail(HJG_EINVAL, "n must be in [1, 48]");
  switch (p->datum) {
    case HJG_L_HALF_SQNORM:
      break;
    case HJG_L_BALL: {
      const double k = p->datum_p[0];
      if (!(k >= 1 && k <= p->n && k == std::floor(k))) return fail(HJG_EINVAL, "ball: datum_p[0] = k in [1, n]");
      if (!std::isfinite(p->datum_p[1])) return fail(HJG_EINVAL, "ball: radius must be finite");
      break;
    }
    case HJG_L_MIN_PAIR_DISKS:
      if (p->n % 3) return fail(HJG_EINVAL, "min_pair_disks needs n = 3m");
      if (!std::isfinite(p->datum_p[0])) return fail(HJG_EINVAL, "radius must be finite");
      break;
    case HJG_L_CAPTURE:
      if (p->n % 3 || p->n < 6 || p->n > 48) return fail(HJG_EINVAL, "capture needs n = 3m, 2 <= m <= 16");
      if (!std::isfinite(p->datum_p[0])) return fail(HJG_EINVAL, "radius must be finite");
      break;
    case HJG_L_KNN_BALLS: {
      const double k = p->datum_p[1];
      if (p->n != 6) return fail(HJG_EINVAL, "knn_balls needs n = 6 (position, velocity)");
      if (!(k >= 1 && k <= kMaxKnn && k == std::floor(k))) return fail(HJG_EINVAL, "knn_balls: K in [1, 8]");
      if (!p->datum_aux) return fail(HJG_EINVAL, "knn_balls needs datum_aux");
      if (!std::isfinite(p->datum_p[0])) return fail(HJG_EINVAL, "radius must be finite");
      break;
    }
    case HJG_L_DISC_UNION: {
      const double k = p->datum_p[1];
      if (p->n < 2 || p->n > 16) return fail(HJG_EINVAL, "disc_union needs 2 <= n <= 16");
      if (!(k >= 1 && k <= kMaxKnn && k == std::floor(k))) return fail(HJG_EINVAL, "disc_union: K in [1, 8]");
      if (!p->datum_aux) return fail(HJG_EINVAL, "disc_union needs datum_aux = centres [K][2]");
      if (!std::isfinite(p->datum_p[0])) return fail(HJG_EINVAL, "radius must be finite");
      break;
    }
    case HJG_L_LINEAR:
      if (!p->datum_aux) return fail(HJG_EINVAL, "linear datum needs datum_aux = a[n]");
      if (!std::isfinite(p->datum_p[0])) return fail(HJG_EINVAL, "offset must be finite");
      break;
    default:
      return fail(HJG_EINVAL, "unknown datum");
  }
  return HJG_OK;
}

DatumP datum_params(const hjg_problem* p) {
  DatumP d;
  d.kind = p->datum;
  d.n = p->n;
  d.k = 0;
  d.m = p->n / 3;
  d.r = 0.f;
  d.aux = p->datum_aux;
  switch (p->datum) {
    case HJG_L_BALL: d.k = (int)p->datum_p[0]; d.r = (float)p->datum_p[1]; break;
    case HJG_L_MIN_PAIR_DISKS: d.r = (float)p->datum_p[0]; break;
    case HJG_L_CAPTURE: d.r = (float)p->datum_p[0]; break;
    case HJG_L_KNN_BALLS: d.r = (float)p->datum_p[0]; d.k = (int)p->datum_p[1]; break;
    case HJG_L_DISC_UNION: d.r = (float)p->datum_p[0]; d.k = (int)p->datum_p[1]; break;
    case HJG_L_LINEAR: d.r = (float)p->datum_p[0]; break;
    default: break;
  }
  return d;
}

HamP ham_params(const hjg_problem* p) {
  HamP h;
  h.kind = p->ham;
  h.n = p->n;
  for (int i = 0; i < 6; ++i) h.p[i] = (float)p->ham_p[i];
  const double delta = 2.0 * p->nu;
  h.inv_delta = (float)(1.0 / delta);
  h.two_over_delta = (float)(2.0 / delta);
  h.eta = (float)p->eta;
  h.c_min = (float)p->c_min;
  h.c_max = (float)p->c_max;
  h.tube = p->tube ? 1 : 0;
  return h;
}

uint32_t make_tag(uint32_t pid, uint32_t step, uint32_t iter) { return (pid << 16) | (step << 8) | iter; }

// The matrix-core pair loop serves bfloat16 common tables with n >= 16
// (HJG_NO_MFMA=1 forces the vector-ALU loop, for comparison).
bool use_mfma(const hjg_problem* p) {
  const char* e = std::getenv("HJG_NO_MFMA");
  if (e && e[0] == '1') return false;
  return p->sample_mode == HJG_S_CRN_STEP && p->sample_bf16 && p->n >= 16 && p->datum != HJG_L_KNN_BALLS &&
         p->datum != HJG_L_DISC_UNION;
}

// Stacked disc pairs on the matrix cores use the one-query-per-lane kernel,
// which reads a float32 sample-major copy of the pair coordinates.
bool pairs_kernel(const hjg_problem* p) { return use_mfma(p) && p->datum == HJG_L_MIN_PAIR_DISKS; }

int queries_per_block(const hjg_problem* p) {
  if (pairs_kernel(p)) return kQueriesPerBlockPairs;
  return use_mfma(p) ? kQueriesPerBlockMfma : kQueriesPerBlockValu;
}

struct Plan {
  int splits;
  int ns;
};

// Cut the N samples of each query into contiguous splits so that the launch
// has enough blocks to fill 256 CUs (about 8 resident blocks each).
int ilog2(int64_t v) {
  int l = 0;
  while (v > 1) { v >>= 1; ++l; }
  return l;
}

// Tuning-table key of a single-problem sweep: kernel specialisation and size bucket.
std::string sweep_key(const hjg_problem* p, int64_t Q, int N) {
  std::ostringstream k;
  k << "sweep " << (use_mfma(p) ? 1 : 0) << ' ' << p->datum << ' ' << n_bucket(p->n) << ' '
    << ((p->datum == HJG_L_MIN_PAIR_DISKS || p->datum == HJG_L_CAPTURE) ? p->n / 3 : 0) << ' ' << p->sample_mode << ' ' << p->sample_bf16 << ' '
    << ilog2(Q) << ' ' << ilog2(N);
  return k.str();
}

// Default number of blocks a sweep launch aims for: the one-query-per-lane
// kernel holds one 8-wave block per CU, so two rounds of blocks (512) keep
// every CU busy with the fewest sample splits; the other kernels run 2 to 4
// smaller blocks per CU.
int default_target_blocks(const hjg_problem* p) { return pairs_kernel(p) ? 512 : 2048; }

// Sample splits for a launch of about `target` blocks.  A split holds at least
// 16 (n + 3) samples: the float64 merge of one state walks its splits
// serially, (n + 3) partials each, so many thin splits of few states would
// make the merge, not the pair loop, the long pole.
Plan plan_splits(int64_t Q, int N, bool fresh, int queries_per_block, int target, int n) {
  if (const char* e = std::getenv("HJG_TARGET_BLOCKS")) target = std::max(1, std::atoi(e));
  const int64_t qblocks = div_up(Q, queries_per_block);
  const int gran = fresh ? 64 : kBlk;
  const int64_t min_ns = div_up(16 * (int64_t)(n + 3), gran) * gran;
  int64_t splits = std::max<int64_t>(1, div_up(target, qblocks));
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, div_up(N, std::max<int64_t>(gran, min_ns))));
  int64_t ns = div_up(div_up(N, splits), gran) * gran;
  splits = div_up(N, ns);
  return Plan{(int)splits, (int)ns};
}

int ensure_partials(hjg_ctx* ctx, int n, int64_t Q, const Plan& pl, bool with_z) {
  const size_t sq = (size_t)pl.splits * (size_t)Q;
  int rc;
  if ((rc = ensure(ctx, ctx->pm, sq * sizeof(float)))) return rc;
  if ((rc = ensure(ctx, ctx->pS, sq * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->pS2, sq * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->pG, sq * n * sizeof(float)))) return rc;
  if (with_z && (rc = ensure(ctx, ctx->pZ, sq * n * sizeof(float)))) return rc;
  return HJG_OK;
}

Partials partials(hjg_ctx* ctx) {
  return Partials{(float*)ctx->pm.p, (double*)ctx->pS.p, (double*)ctx->pS2.p, (float*)ctx->pG.p, (float*)ctx->pZ.p};
}

// The common table of (problem, time step), generated on the caller's stream
// unless the cached one matches; its column mean too when cv is requested.
int ensure_table(hjg_ctx* ctx, const hjg_problem* p, int N, uint32_t step, bool need_zbar, hipStream_t s) {
  const bool bf16 = p->sample_bf16 != 0;
  const int64_t tstride = div_up(N, 64) * 64;
  const bool zd = pairs_kernel(p);
  const bool hit = ctx->table_valid && ctx->t_seed == p->seed && ctx->t_pid == p->problem_id &&
                   ctx->t_step == step && ctx->t_n == p->n && ctx->t_N == N && ctx->t_bf16 == (int)bf16 &&
                   (!zd || ctx->t_zd);
  int rc;
  if (!hit) {
    const int64_t tbytes = (int64_t)p->n * tstride * (bf16 ? 2 : 4);
    const int64_t zoff = (tbytes + 255) / 256 * 256;
    const int zs = pair_coord_stride(p->n / 3);
    if ((rc = ensure(ctx, ctx->table, zd ? (size_t)(zoff + (int64_t)N * zs * 4) : (size_t)tbytes))) return rc;
    const uint32_t k0 = (uint32_t)(p->seed & 0xFFFFFFFFu), k1 = (uint32_t)(p->seed >> 32);
    HJG_HIP(launch_table(p->n, tstride, tstride, k0, k1, make_tag(p->problem_id, step, 0), bf16, ctx->table.p, s));
    if (zd) HJG_HIP(launch_pair_coords(p->n / 3, N, tstride, ctx->table.p, zs, (float*)((char*)ctx->table.p + zoff), s));
    ctx->t_zd = zd;
    ctx->t_zoff = zoff;
    ctx->table_valid = true;
    ctx->t_seed = p->seed;
    ctx->t_pid = p->problem_id;
    ctx->t_step = step;
    ctx->t_n = p->n;
    ctx->t_N = N;
    ctx->t_bf16 = bf16;
    ctx->t_stride = tstride;
    ctx->zbar_valid = 0;
  }
  if (need_zbar && !ctx->zbar_valid) {
    if ((rc = ensure(ctx, ctx->zbar, kMaxN * sizeof(double)))) return rc;
    HJG_HIP(launch_zbar(p->n, N, ctx->t_stride, bf16, ctx->table.p, (double*)ctx->zbar.p, s));
    ctx->zbar_valid = 1;
  }
  return HJG_OK;
}

const float* table_zd(const hjg_ctx* ctx, const hjg_problem* p) {
  return pairs_kernel(p) && ctx->t_zd ? (const float*)((const char*)ctx->table.p + ctx->t_zoff) : nullptr;
}

int ensure_events(hjg_ctx* ctx) {
  if (!ctx->ev.empty()) return HJG_OK;
  ctx->ev.resize(2 * kMaxTimed, nullptr);
  for (auto& e : ctx->ev) HJG_HIP(hipEventCreate(&e));
  return HJG_OK;
}

int check_common(hjg_ctx* ctx, const hjg_problem* p, int64_t Q, double t, int32_t N, uint32_t step) {
  if (!ctx) return fail(HJG_EINVAL, "context is NULL");
  int rc = check_problem(p);
  if (rc) return rc;
  if (Q < 0 || Q > (int64_t)1 << 30) return fail(HJG_EINVAL, "Q must be in [0, 2^30]");
  if (!finite_pos(t)) return fail(HJG_EINVAL, "t must be finite and > 0");
  if (N < 1 || N > (1 << 30)) return fail(HJG_EINVAL, "N must be in [1, 2^30]");
  if (step >= 256) return fail(HJG_EINVAL, "time_step must be < 256");
  return HJG_OK;
}

}  // namespace

namespace hjg {
namespace detail {
int check_problem(const hjg_problem* p) { return ::check_problem(p); }
int check_datum(const hjg_problem* p) { return ::check_datum(p); }
DatumP datum_params(const hjg_problem* p) { return ::datum_params(p); }
HamP ham_params(const hjg_problem* p) { return ::ham_params(p); }
uint32_t make_tag(uint32_t pid, uint32_t step, uint32_t iter) { return ::make_tag(pid, step, iter); }
}  // namespace detail
}  // namespace hjg

extern "C" {

// Error reporting shared with the other translation units of the library.
__attribute__((visibility("hidden"))) int hjg_internal_fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

const char* hjg_last_error(void) { return g_err.c_str(); }

const char* hjg_version(void) { return "hjg 0.1 (gfx950)"; }

int hjg_ctx_create(int device, hjg_ctx** out) {
  g_err.clear();
  if (!out) return fail(HJG_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  HJG_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(HJG_EINVAL, "device index out of range");
  HJG_HIP(hipSetDevice(device));
  if (device >= kMaxDevices) return fail(HJG_EINVAL, "device index above 63");
  void* scr = nullptr;
  {
    // once per device, with that device current: the address of this
    // device's copy of the scratch array
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(HJG_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
      g_scratch_ptr[device] = p;
    }
    scr = g_scratch_ptr[device];
  }
  hjg_ctx* ctx = new hjg_ctx();
  ctx->device = device;
  ctx->scratch = scr;
  if (hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return fail(HJG_EHIP, "cannot create the graph-recording stream");
  }
  *out = ctx;
  return HJG_OK;
}

void hjg_ctx_destroy(hjg_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  drop_graphs(ctx);
  for (DevBuf* b : {&ctx->pm, &ctx->pS, &ctx->pS2, &ctx->pG, &ctx->pZ, &ctx->vprev, &ctx->cwork, &ctx->thwork,
                    &ctx->blockpart, &ctx->resid, &ctx->ctrl, &ctx->table, &ctx->zbar, &ctx->batch.ws,
                    &ctx->batch.args, &ctx->batch.items, &ctx->g_cell, &ctx->g_rank, &ctx->g_start, &ctx->g_bsum,
                    &ctx->g_sorted})
    if (b->p) (void)hipFree(b->p);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (int j = 0; j < hjg_ctx::kSide; ++j) {
    if (ctx->side[j]) (void)hipStreamDestroy(ctx->side[j]);
    if (ctx->join_ev[j]) (void)hipEventDestroy(ctx->join_ev[j]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->batch.replay_ev) (void)hipEventDestroy(ctx->batch.replay_ev);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
}

int hjg_philox4x32_10(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t G, uint32_t* out,
                      void* hip_stream) {
  g_err.clear();
  if (G < 0) return fail(HJG_EINVAL, "G must be >= 0");
  if (G == 0) return HJG_OK;
  if (!out) return fail(HJG_EINVAL, "out is NULL");
  HJG_HIP(launch_philox_words((uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), c1, c2, c3, G, out,
                              (hipStream_t)hip_stream));
  return HJG_OK;
}

int hjg_sample_table(hjg_ctx* ctx, const hjg_problem* p, int32_t N, uint32_t step, void* out, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_sample_table");
  g_err.clear();
  int rc = check_common(ctx, p, 0, 1.0, N, step);
  if (rc) return rc;
  if (!out) return fail(HJG_EINVAL, "out is NULL");
  HJG_HIP(hipSetDevice(ctx->device));
  const uint32_t k0 = (uint32_t)(p->seed & 0xFFFFFFFFu), k1 = (uint32_t)(p->seed >> 32);
  HJG_HIP(launch_table(p->n, N, N, k0, k1, make_tag(p->problem_id, step, 0), p->sample_bf16 != 0, out,
                       (hipStream_t)hip_stream));
  return HJG_OK;
}

int hjg_value_grad(hjg_ctx* ctx, const hjg_problem* p, int64_t Q, const float* x, double t, int32_t N,
                   uint32_t step, uint32_t iter, const float* c, const float* theta, float* v, float* grad,
                   float* ess, int32_t check_finite, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_value_grad");
  g_err.clear();
  int rc = check_common(ctx, p, Q, t, N, step);
  if (rc) return rc;
  if (iter >= 256) return fail(HJG_EINVAL, "iter must be < 256");
  if (Q == 0) return HJG_OK;
  if (!x || !c || !v || !grad) return fail(HJG_EINVAL, "x, c, v and grad are required");
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool fresh = p->sample_mode == HJG_S_FRESH;
  const bool mf = use_mfma(p);
  const auto tv = ctx->tuning.find(sweep_key(p, Q, N));
  const Plan pl = plan_splits(Q, N, fresh, queries_per_block(p),
                              tv == ctx->tuning.end() ? default_target_blocks(p) : tv->second, p->n);
  if ((rc = ensure_partials(ctx, p->n, Q, pl, fresh && p->grad_cv))) return rc;
  if (!fresh && (rc = ensure_table(ctx, p, N, step, p->grad_cv != 0, s))) return rc;
  const float sigma = (float)std::sqrt(2.0 * p->nu * t);

  SweepArgs a{};
  a.n = p->n;
  a.Q = Q;
  a.N = N;
  a.ns = pl.ns;
  a.splits = pl.splits;
  a.x = x;
  a.c = c;
  a.theta = theta;
  a.sigma = sigma;
  a.table = fresh ? nullptr : ctx->table.p;
  a.tstride = ctx->t_stride;
  a.zd = fresh ? nullptr : table_zd(ctx, p);
  a.dp = datum_params(p);
  a.k0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(p->seed >> 32);
  a.tag = make_tag(p->problem_id, step, iter);
  a.cv = p->grad_cv;
  a.mfma = mf;
  a.part = partials(ctx);
  a.done = nullptr;
  if (ctx->timing) {
    if ((rc = ensure_events(ctx))) return rc;
    HJG_HIP(hipEventRecord(ctx->ev[0], s));
  }
  HJG_HIP(launch_sweep(a, fresh, p->sample_bf16 != 0, s));
  if (ctx->timing) {
    HJG_HIP(hipEventRecord(ctx->ev[1], s));
    ctx->last_pairs = 1;
  }

  FinalizeArgs f{};
  f.n = p->n;
  f.Q = Q;
  f.N = N;
  f.splits = pl.splits;
  f.sigma = sigma;
  f.x = x;
  f.c = c;
  f.theta = theta;
  f.part = a.part;
  f.cv = p->grad_cv;
  f.fresh = fresh;
  f.zbar_tab = (const double*)ctx->zbar.p;
  f.v = v;
  f.grad = grad;
  f.ess = ess;
  f.picard = 0;
  f.hp = ham_params(p);
  HJG_HIP(launch_finalize(f, s));

  if (check_finite) {
    if ((rc = ensure(ctx, ctx->ctrl, kCtrlWords * sizeof(int)))) return rc;
    int* flag = (int*)ctx->ctrl.p + 2;
    HJG_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    HJG_HIP(launch_finite_check(v, Q, flag, s));
    HJG_HIP(launch_finite_check(grad, Q * p->n, flag, s));
    int host = 0;
    HJG_HIP(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HJG_HIP(hipStreamSynchronize(s));
    if (host) return fail(HJG_ENONFINITE, "non-finite value in v or grad");
  }
  return HJG_OK;
}

int hjg_value_grad_noalloc(hjg_ctx* ctx, const hjg_problem* p, int64_t Q, const float* x, double t, int32_t N,
                           uint32_t step, uint32_t iter, const float* c, const float* theta, float* v, float* grad,
                           float* ess, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_value_grad_noalloc");
  g_err.clear();
  int rc = check_common(ctx, p, Q, t, N, step);
  if (rc) return rc;
  if (iter >= 256) return fail(HJG_EINVAL, "iter must be < 256");
  if (Q == 0) return HJG_OK;
  if (!x || !c || !v || !grad) return fail(HJG_EINVAL, "x, c, v and grad are required");
  if (!ctx->scratch) return fail(HJG_EINVAL, "the context has no scratch address");
  const bool fresh = p->sample_mode == HJG_S_FRESH;
  const bool bf16 = p->sample_bf16 != 0;
  const bool zdc = !fresh && pairs_kernel(p);
  const auto tv = ctx->tuning.find(sweep_key(p, Q, N));
  const Plan pl = plan_splits(Q, N, fresh, queries_per_block(p),
                              tv == ctx->tuning.end() ? default_target_blocks(p) : tv->second, p->n);
  // carve the scratch exactly as the allocating entry point sizes its buffers
  const int64_t tstride = div_up(N, 64) * 64;
  const int64_t sq = (int64_t)pl.splits * Q;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const int64_t o_m = take(sq * 4), o_S = take(sq * 8), o_S2 = take(sq * 8), o_G = take(sq * p->n * 4);
  const int64_t o_Z = fresh && p->grad_cv ? take(sq * p->n * 4) : -1;
  const int64_t o_tab = fresh ? -1 : take((int64_t)p->n * tstride * (bf16 ? 2 : 4));
  const int64_t o_zd = zdc ? take((int64_t)N * pair_coord_stride(p->n / 3) * 4) : -1;
  const int64_t o_zb = !fresh && p->grad_cv ? take(kMaxN * 8) : -1;
  if (off > (int64_t)kNoallocScratchBytes)
    return fail(HJG_EINVAL, "needs " + std::to_string(off) + " bytes of scratch, more than the " +
                                std::to_string(kNoallocScratchBytes) + " available (reduce Q or N)");
  char* base = (char*)ctx->scratch;
  auto at = [&](int64_t o) -> void* { return o < 0 ? nullptr : (void*)(base + o); };
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  if (!fresh) {
    const uint32_t k0 = (uint32_t)(p->seed & 0xFFFFFFFFu), k1 = (uint32_t)(p->seed >> 32);
    HJG_HIP(launch_table(p->n, tstride, tstride, k0, k1, make_tag(p->problem_id, step, 0), bf16, at(o_tab), s));
    if (zdc)
      HJG_HIP(launch_pair_coords(p->n / 3, N, tstride, at(o_tab), pair_coord_stride(p->n / 3), (float*)at(o_zd), s));
    if (p->grad_cv) HJG_HIP(launch_zbar(p->n, N, tstride, bf16, at(o_tab), (double*)at(o_zb), s));
  }
  const float sigma = (float)std::sqrt(2.0 * p->nu * t);
  const Partials part{(float*)at(o_m), (double*)at(o_S), (double*)at(o_S2), (float*)at(o_G), (float*)at(o_Z)};

  SweepArgs a{};
  a.n = p->n;
  a.Q = Q;
  a.N = N;
  a.ns = pl.ns;
  a.splits = pl.splits;
  a.x = x;
  a.c = c;
  a.theta = theta;
  a.sigma = sigma;
  a.table = at(o_tab);
  a.tstride = tstride;
  a.zd = (const float*)at(o_zd);
  a.dp = datum_params(p);
  a.k0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(p->seed >> 32);
  a.tag = make_tag(p->problem_id, step, iter);
  a.cv = p->grad_cv;
  a.mfma = use_mfma(p);
  a.part = part;
  a.done = nullptr;
  HJG_HIP(launch_sweep(a, fresh, bf16, s));

  FinalizeArgs f{};
  f.n = p->n;
  f.Q = Q;
  f.N = N;
  f.splits = pl.splits;
  f.sigma = sigma;
  f.x = x;
  f.c = c;
  f.theta = theta;
  f.part = part;
  f.cv = p->grad_cv;
  f.fresh = fresh;
  f.zbar_tab = (const double*)at(o_zb);
  f.v = v;
  f.grad = grad;
  f.ess = ess;
  f.picard = 0;
  f.hp = ham_params(p);
  HJG_HIP(launch_finalize(f, s));
  return HJG_OK;
}

namespace {

// Everything a recorded Picard graph depends on.
struct PicardKey {
  hjg_problem p;
  int64_t Q;
  const float* x;
  double t;
  int32_t N, K;
  double tol;
  uint32_t step;
  const float *p0, *v0;
  float *v, *grad, *c_out, *ess;
  uint8_t* flags;
  void* table;
  int splits, ns;
  int timing;
  int mfma;
};

// Field-by-field copy into zeroed storage so padding bytes never differ.
void copy_problem(hjg_problem* dst, const hjg_problem* src) {
  std::memset(dst, 0, sizeof(*dst));
  dst->n = src->n;
  dst->ham = src->ham;
  dst->datum = src->datum;
  for (int i = 0; i < 8; ++i) dst->ham_p[i] = src->ham_p[i];
  for (int i = 0; i < 4; ++i) dst->datum_p[i] = src->datum_p[i];
  dst->datum_aux = src->datum_aux;
  dst->nu = src->nu;
  dst->eta = src->eta;
  dst->c_min = src->c_min;
  dst->c_max = src->c_max;
  dst->tilt = src->tilt;
  dst->sample_mode = src->sample_mode;
  dst->sample_bf16 = src->sample_bf16;
  dst->grad_cv = src->grad_cv;
  dst->seed = src->seed;
  dst->problem_id = src->problem_id;
  dst->tube = src->tube;
}

int record_picard(hjg_ctx* ctx, const PicardKey& k, hipStream_t s) {
  const hjg_problem* p = &k.p;
  const bool fresh = p->sample_mode == HJG_S_FRESH;
  const float sigma = (float)std::sqrt(2.0 * p->nu * k.t);
  const int64_t Q = k.Q;
  const int nblocks = (int)div_up(Q, kThreads);
  int* done = (int*)ctx->ctrl.p;
  int* iters = done + 1;
  int* nonfinite = done + kCtrlNonfinite;
  float* th = p->tilt ? (float*)ctx->thwork.p : nullptr;

  InitArgs in{};
  in.n = p->n;
  in.Q = Q;
  in.K = k.K;
  in.sigma = sigma;
  in.x = k.x;
  in.p0 = k.p0;
  in.v0 = k.v0;
  in.dp = datum_params(p);
  in.hp = ham_params(p);
  in.tilt = p->tilt;
  in.vprev = (float*)ctx->vprev.p;
  in.p = k.grad;
  in.c = (float*)ctx->cwork.p;
  in.th = th;
  in.done = done;
  in.iters = iters;
  in.nonfinite = nonfinite;
  in.resid = (double*)ctx->resid.p;
  HJG_HIP(launch_init(in, s));

  for (int it = 0; it < k.K; ++it) {
    SweepArgs a{};
    a.n = p->n;
    a.Q = Q;
    a.N = k.N;
    a.ns = k.ns;
    a.splits = k.splits;
    a.x = k.x;
    a.c = (const float*)ctx->cwork.p;
    a.theta = th;
    a.sigma = sigma;
    a.table = fresh ? nullptr : ctx->table.p;
    a.tstride = ctx->t_stride;
    a.zd = fresh ? nullptr : table_zd(ctx, p);
    a.dp = in.dp;
    a.k0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(p->seed >> 32);
    a.tag = make_tag(p->problem_id, k.step, fresh ? (uint32_t)it : 0u);
    a.cv = p->grad_cv;
    a.mfma = use_mfma(p);
    a.part = partials(ctx);
    a.done = done;
    if (k.timing) HJG_HIP(hipEventRecord(ctx->ev[2 * it], s));
    HJG_HIP(launch_sweep(a, fresh, p->sample_bf16 != 0, s));
    if (k.timing) HJG_HIP(hipEventRecord(ctx->ev[2 * it + 1], s));

    FinalizeArgs f{};
    f.n = p->n;
    f.Q = Q;
    f.N = k.N;
    f.splits = k.splits;
    f.sigma = sigma;
    f.x = k.x;
    f.c = (const float*)ctx->cwork.p;
    f.theta = th;
    f.part = a.part;
    f.cv = p->grad_cv;
    f.fresh = fresh;
    f.zbar_tab = (const double*)ctx->zbar.p;
    f.v = k.v;
    f.grad = k.grad;
    f.ess = k.ess;
    f.picard = 1;
    f.vprev = (float*)ctx->vprev.p;
    f.c_out = k.c_out;
    f.flags = k.flags;
    f.tol = (float)k.tol;
    f.vfloor = (float)(1e-2 * std::sqrt(2.0 * p->nu * k.t) * std::sqrt((double)p->n));
    f.blockpart = (double*)ctx->blockpart.p;
    f.c_next = (float*)ctx->cwork.p;
    f.th_next = th;
    f.hp = in.hp;
    f.done = done;
    HJG_HIP(launch_finalize(f, s));

    ReduceArgs r{};
    r.nblocks = nblocks;
    r.blockpart = (const double*)ctx->blockpart.p;
    r.k = it;
    r.tol = (float)k.tol;
    r.resid = (double*)ctx->resid.p;
    r.done = done;
    r.iters = iters;
    r.nonfinite = nonfinite;
    HJG_HIP(launch_reduce(r, s));
  }
  return HJG_OK;
}

}  // namespace

int hjg_picard_sweep(hjg_ctx* ctx, const hjg_problem* p, int64_t Q, const float* x, double t, int32_t N, int32_t K,
                     double tol, uint32_t step, const float* p0, const float* v0, float* v, float* grad,
                     float* c_out, float* ess, uint8_t* flags, double* resid_hist, int32_t* iters_done,
                     void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_picard_sweep");
  g_err.clear();
  int rc = check_common(ctx, p, Q, t, N, step);
  if (rc) return rc;
  if (K < 1 || K > 255) return fail(HJG_EINVAL, "K must be in [1, 255]");
  if (!std::isfinite(tol)) return fail(HJG_EINVAL, "tol must be finite");
  if (Q == 0) {
    if (iters_done) *iters_done = 0;
    if (resid_hist) std::fill(resid_hist, resid_hist + K, 0.0);
    return HJG_OK;
  }
  if (!x || !v || !grad) return fail(HJG_EINVAL, "x, v and grad are required");
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool fresh = p->sample_mode == HJG_S_FRESH;
  const auto tv = ctx->tuning.find(sweep_key(p, Q, N));
  const Plan pl = plan_splits(Q, N, fresh, queries_per_block(p),
                              tv == ctx->tuning.end() ? default_target_blocks(p) : tv->second, p->n);
  if ((rc = ensure_partials(ctx, p->n, Q, pl, fresh && p->grad_cv))) return rc;
  if ((rc = ensure(ctx, ctx->vprev, Q * sizeof(float)))) return rc;
  if ((rc = ensure(ctx, ctx->cwork, Q * sizeof(float)))) return rc;
  if (p->tilt && (rc = ensure(ctx, ctx->thwork, (size_t)Q * p->n * sizeof(float)))) return rc;
  if ((rc = ensure(ctx, ctx->blockpart, (size_t)div_up(Q, kThreads) * 3 * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->resid, 256 * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->ctrl, kCtrlWords * sizeof(int)))) return rc;
  if (!fresh && (rc = ensure_table(ctx, p, N, step, p->grad_cv != 0, s))) return rc;

  PicardKey key;
  std::memset(&key, 0, sizeof(key));
  copy_problem(&key.p, p);
  key.Q = Q;
  key.x = x;
  key.t = t;
  key.N = N;
  key.K = K;
  key.tol = tol;
  key.step = step;
  key.p0 = p0;
  key.v0 = v0;
  key.v = v;
  key.grad = grad;
  key.c_out = c_out;
  key.ess = ess;
  key.flags = flags;
  key.table = fresh ? nullptr : ctx->table.p;
  key.splits = pl.splits;
  key.ns = pl.ns;
  key.timing = ctx->timing;
  key.mfma = use_mfma(p);
  if (ctx->timing) {
    if ((rc = ensure_events(ctx))) return rc;
    ctx->last_pairs = K;
  }

  // With timing on, launch kernel by kernel: HIP cannot take elapsed times
  // from events recorded as nodes of a graph.
  const char* ng = std::getenv("HJG_NO_GRAPH");
  if ((ng && ng[0] == '1') || ctx->timing) {
    if ((rc = record_picard(ctx, key, s))) return rc;
  } else {
    std::vector<char> kb(sizeof(key));
    std::memcpy(kb.data(), &key, sizeof(key));
    hjg_ctx::Graph* found = nullptr;
    for (auto& g : ctx->graphs)
      if (g.key == kb) found = &g;
    if (!found) {
      if (ctx->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        (void)hipGraphDestroy(ctx->graphs.front().graph);
        ctx->graphs.erase(ctx->graphs.begin());
      }
      HJG_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
      rc = record_picard(ctx, key, ctx->cap);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) return fail(HJG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      hipGraphExec_t exec = nullptr;
      const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(HJG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
      }
      ctx->graphs.push_back(hjg_ctx::Graph{kb, graph, exec});
      found = &ctx->graphs.back();
    }
    HJG_HIP(hipGraphLaunch(found->exec, s));
  }

  if (resid_hist || iters_done || tol > 0) {
    int ctrl[kCtrlWords] = {};
    HJG_HIP(hipMemcpyAsync(ctrl, ctx->ctrl.p, sizeof(ctrl), hipMemcpyDeviceToHost, s));
    if (resid_hist) HJG_HIP(hipMemcpyAsync(resid_hist, ctx->resid.p, K * sizeof(double), hipMemcpyDeviceToHost, s));
    HJG_HIP(hipStreamSynchronize(s));
    if (iters_done) *iters_done = ctrl[1];
    if (ctrl[kCtrlNonfinite])
      return fail(HJG_ENONFINITE, std::to_string(ctrl[kCtrlNonfinite]) + " of " + std::to_string(Q) +
                                      " states have a non-finite value or gradient after iteration " +
                                      std::to_string(ctrl[1]));
    if (tol > 0 && !ctrl[0]) {
      g_err = "tolerance not reached within K iterations";
      return HJG_ENOTCONVERGED;
    }
  }
  return HJG_OK;
}

int hjg_set_timing(hjg_ctx* ctx, int32_t enable) {
  g_err.clear();
  if (!ctx) return fail(HJG_EINVAL, "context is NULL");
  HJG_HIP(hipSetDevice(ctx->device));
  if (enable) {
    const int rc = ensure_events(ctx);
    if (rc) return rc;
  }
  ctx->timing = enable ? 1 : 0;
  ctx->last_pairs = 0;
  return HJG_OK;
}

int hjg_sweep_time(hjg_ctx* ctx, double* total_ms, int32_t* launches) {
  g_err.clear();
  if (!ctx || !total_ms || !launches) return fail(HJG_EINVAL, "NULL argument");
  *total_ms = 0.0;
  *launches = 0;
  if (!ctx->timing || ctx->last_pairs == 0) return HJG_OK;
  HJG_HIP(hipSetDevice(ctx->device));
  HJG_HIP(hipEventSynchronize(ctx->ev[2 * ctx->last_pairs - 1]));
  for (int i = 0; i < ctx->last_pairs; ++i) {
    float ms = 0.f;
    HJG_HIP(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
    *total_ms += ms;
  }
  *launches = ctx->last_pairs;
  return HJG_OK;
}

}  // extern "C"

// ===================================================================== batched
namespace {

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// Kernel specialisation of a problem's pair loop (problems that share it can
// share a launch).
struct SpecKey {
  int datum, bucket, pairs, mfma, bf16;
  bool operator<(const SpecKey& o) const {
    return std::tie(datum, bucket, pairs, mfma, bf16) < std::tie(o.datum, o.bucket, o.pairs, o.mfma, o.bf16);
  }
};

// Samples per split in a batched launch: the batch as a whole fills the GPU,
// so each problem is cut only into splits of about this many samples.
// Launch mode of a batch, bit 0: persistent launches (resident blocks take
// work items from a queue) rather than one block per item; bit 1: the chains
// of the kernel specialisations (each its problems' levels in order) as
// parallel branches of the recorded graph rather than one after another.  Default both; the tuning entry "batch_mode" holds the
// autotuner's choice as mode + 1; HJG_BATCH_PERSISTENT / HJG_BATCH_CONCURRENT
// = 0 or 1 override a bit.
int batched_mode(const hjg_ctx* ctx) {
  int mode = 3;
  const auto it = ctx->tuning.find("batch_mode");
  if (it != ctx->tuning.end() && it->second >= 1 && it->second <= 4) mode = it->second - 1;
  if (const char* e = std::getenv("HJG_BATCH_PERSISTENT")) mode = e[0] == '0' ? (mode & ~1) : (mode | 1);
  if (const char* e = std::getenv("HJG_BATCH_CONCURRENT")) mode = e[0] == '0' ? (mode & ~2) : (mode | 2);
  return mode;
}

int ensure_side(hjg_ctx* ctx) {
  if (ctx->fork_ev) return HJG_OK;
  for (int j = 0; j < hjg_ctx::kSide; ++j) {
    HJG_HIP(hipStreamCreateWithFlags(&ctx->side[j], hipStreamNonBlocking));
    HJG_HIP(hipEventCreateWithFlags(&ctx->join_ev[j], hipEventDisableTiming));
  }
  HJG_HIP(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  return HJG_OK;
}

int batched_split_samples(const hjg_ctx* ctx) {
  int ns = 4096;
  const auto it = ctx->tuning.find("batch");
  if (it != ctx->tuning.end()) ns = it->second;
  if (const char* e = std::getenv("HJG_BATCH_SPLIT")) ns = std::atoi(e);
  ns = std::max(ns, kBlk);
  return ns / kBlk * kBlk;
}

}  // namespace

extern "C" int hjg_picard_sweep_batched(hjg_ctx* ctx, int32_t P, const hjg_problem* probs, const int64_t* q_off,
                                        const int32_t* Ns, const int32_t* Ks, const double* ts, double tol,
                                        const float* x_all, float* v_all, float* grad_all, double* resid_hist,
                                        int32_t* iters, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_picard_sweep_batched");
  g_err.clear();
  if (!ctx || !probs || !q_off || !Ns || !Ks || !ts) return fail(HJG_EINVAL, "NULL argument");
  if (P < 1 || P > 65536) return fail(HJG_EINVAL, "P must be in [1, 65536]");
  if (!std::isfinite(tol)) return fail(HJG_EINVAL, "tol must be finite");
  if (q_off[0] != 0) return fail(HJG_EINVAL, "q_off[0] must be 0");
  int Kmax = 0;
  std::vector<int64_t> xo(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    const int64_t Q = q_off[p + 1] - q_off[p];
    int rc = check_common(ctx, &probs[p], Q, ts[p], Ns[p], 0);
    if (rc) return fail(rc, "problem " + std::to_string(p) + ": " + g_err);
    if (Q < 1) return fail(HJG_EINVAL, "problem " + std::to_string(p) + ": needs at least one state");
    if (probs[p].sample_mode != HJG_S_CRN_STEP)
      return fail(HJG_EUNSUPPORTED, "batched sweeps use common-random-number tables");
    if (Ks[p] < 1 || Ks[p] > 255) return fail(HJG_EINVAL, "K must be in [1, 255]");
    Kmax = std::max(Kmax, (int)Ks[p]);
    xo[p + 1] = xo[p] + Q * probs[p].n;
  }
  if (!x_all || !v_all || !grad_all) return fail(HJG_EINVAL, "x_all, v_all and grad_all are required");
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  auto& B = ctx->batch;

  // ---- key of this batch: every input the recorded graph depends on
  std::vector<char> key;
  auto put = [&](const void* d, size_t n) { key.insert(key.end(), (const char*)d, (const char*)d + n); };
  put(&P, sizeof(P));
  for (int p = 0; p < P; ++p) {
    hjg_problem c;
    copy_problem(&c, &probs[p]);
    put(&c, sizeof(c));
  }
  put(q_off, sizeof(int64_t) * (P + 1));
  put(Ns, sizeof(int32_t) * P);
  put(Ks, sizeof(int32_t) * P);
  put(ts, sizeof(double) * P);
  put(&tol, sizeof(tol));
  put(&x_all, sizeof(x_all));
  put(&v_all, sizeof(v_all));
  put(&grad_all, sizeof(grad_all));
  const int split_ns = batched_split_samples(ctx);
  put(&split_ns, sizeof(split_ns));
  const int mode = batched_mode(ctx);
  put(&mode, sizeof(mode));

  if (key != B.key || !B.exec) {
    // a replay of the previous plan may still run on some stream: it reads
    // the buffers rewritten below
    if (!B.replay_ev) HJG_HIP(hipEventCreateWithFlags(&B.replay_ev, hipEventDisableTiming));
    else HJG_HIP(hipEventSynchronize(B.replay_ev));
    drop_batch_graph(ctx);
    // ---- per-problem plan and workspace carving
    struct Plan1 {
      int64_t Q, qb_sweep, qb256;
      int splits, ns, mfma, bf16;
      int64_t tstride;
      int64_t o_m, o_S, o_S2, o_G, o_vp, o_c, o_th, o_bp, o_res, o_ctrl, o_tab, o_zb, o_zd;
    };
    std::vector<Plan1> pl(P);
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
      const int64_t o = off;
      off += align256(std::max<int64_t>(bytes, 8));
      return o;
    };
    for (int p = 0; p < P; ++p) {
      const hjg_problem& pr = probs[p];
      Plan1& q = pl[p];
      q.Q = q_off[p + 1] - q_off[p];
      q.mfma = use_mfma(&pr);
      q.bf16 = pr.sample_bf16 != 0;
      const int qpb = queries_per_block(&pr);
      q.qb_sweep = div_up(q.Q, qpb);
      q.qb256 = div_up(q.Q, kThreads);
      q.ns = std::min<int64_t>(split_ns, div_up(Ns[p], kBlk) * kBlk);
      q.splits = (int)div_up(Ns[p], q.ns);
      q.tstride = div_up(Ns[p], 64) * 64;
      const int64_t sq = (int64_t)q.splits * q.Q;
      q.o_m = take(sq * 4);
      q.o_S = take(sq * 8);
      q.o_S2 = take(sq * 8);
      q.o_G = take(sq * pr.n * 4);
      q.o_vp = take(q.Q * 4);
      q.o_c = take(q.Q * 4);
      q.o_th = pr.tilt ? take(q.Q * pr.n * 4) : -1;
      q.o_bp = take(q.qb256 * 24);
      q.o_res = take(Ks[p] * 8);
      q.o_ctrl = take(16);
      q.o_tab = take((int64_t)pr.n * q.tstride * (q.bf16 ? 2 : 4));
      q.o_zb = pr.grad_cv ? take(pr.n * 8) : -1;
      q.o_zd = pairs_kernel(&pr) ? take((int64_t)Ns[p] * pair_coord_stride(pr.n / 3) * 4) : -1;
    }
    int rc;
    if ((rc = ensure(ctx, B.ws, off))) return rc;
    char* ws = (char*)B.ws.p;
    auto at = [&](int64_t o) -> void* { return o < 0 ? nullptr : (void*)(ws + o); };

    // ---- argument records
    std::vector<SweepArgs> sa(P);
    std::vector<FinalizeArgs> fa(P);
    std::vector<InitArgs> ia(P);
    std::vector<ReduceArgs> ra(P);
    B.resid_off.assign(P, 0);
    B.ctrl_off.assign(P, 0);
    B.K.assign(Ks, Ks + P);
    for (int p = 0; p < P; ++p) {
      const hjg_problem& pr = probs[p];
      const Plan1& q = pl[p];
      const float sigma = (float)std::sqrt(2.0 * pr.nu * ts[p]);
      int* done = (int*)at(q.o_ctrl);
      const Partials part{(float*)at(q.o_m), (double*)at(q.o_S), (double*)at(q.o_S2), (float*)at(q.o_G), nullptr};
      float* th = (float*)at(q.o_th);
      SweepArgs& A = sa[p];
      A = SweepArgs{};
      A.n = pr.n;
      A.Q = q.Q;
      A.N = Ns[p];
      A.ns = q.ns;
      A.splits = q.splits;
      A.x = x_all + xo[p];
      A.c = (const float*)at(q.o_c);
      A.theta = th;
      A.sigma = sigma;
      A.table = at(q.o_tab);
      A.tstride = q.tstride;
      A.zd = (const float*)at(q.o_zd);
      A.dp = datum_params(&pr);
      A.k0 = (uint32_t)(pr.seed & 0xFFFFFFFFu);
      A.k1 = (uint32_t)(pr.seed >> 32);
      A.cv = pr.grad_cv;
      A.mfma = q.mfma;
      A.part = part;
      A.done = done;
      FinalizeArgs& F = fa[p];
      F = FinalizeArgs{};
      F.n = pr.n;
      F.Q = q.Q;
      F.N = Ns[p];
      F.splits = q.splits;
      F.sigma = sigma;
      F.x = A.x;
      F.c = A.c;
      F.theta = th;
      F.part = part;
      F.cv = pr.grad_cv;
      F.fresh = 0;
      F.zbar_tab = (const double*)at(q.o_zb);
      F.v = v_all + q_off[p];
      F.grad = grad_all + xo[p];
      F.ess = nullptr;
      F.picard = 1;
      F.vprev = (float*)at(q.o_vp);
      F.tol = (float)tol;
      F.vfloor = (float)(1e-2 * std::sqrt(2.0 * pr.nu * ts[p]) * std::sqrt((double)pr.n));
      F.blockpart = (double*)at(q.o_bp);
      F.c_next = (float*)at(q.o_c);
      F.th_next = th;
      F.hp = ham_params(&pr);
      F.done = done;
      InitArgs& I = ia[p];
      I = InitArgs{};
      I.n = pr.n;
      I.Q = q.Q;
      I.K = Ks[p];
      I.sigma = sigma;
      I.x = A.x;
      I.dp = A.dp;
      I.hp = F.hp;
      I.tilt = pr.tilt;
      I.vprev = F.vprev;
      I.p = F.grad;
      I.c = (float*)at(q.o_c);
      I.th = th;
      I.done = done;
      I.iters = done + 1;
      I.nonfinite = done + 2;
      I.resid = (double*)at(q.o_res);
      ReduceArgs& R = ra[p];
      R = ReduceArgs{};
      R.nblocks = (int)q.qb256;
      R.blockpart = F.blockpart;
      R.tol = (float)tol;
      R.resid = I.resid;
      R.done = done;
      R.iters = done + 1;
      R.nonfinite = done + 2;
      B.resid_off[p] = q.o_res;
      B.ctrl_off[p] = q.o_ctrl;
    }
    const int64_t o_sa = 0, o_fa = align256(P * sizeof(SweepArgs));
    const int64_t o_ia = o_fa + align256(P * sizeof(FinalizeArgs));
    const int64_t o_ra = o_ia + align256(P * sizeof(InitArgs));
    const int64_t args_bytes = o_ra + align256(P * sizeof(ReduceArgs));
    if ((rc = ensure(ctx, B.args, args_bytes))) return rc;
    char* ab = (char*)B.args.p;
    HJG_HIP(hipMemcpy(ab + o_sa, sa.data(), P * sizeof(SweepArgs), hipMemcpyHostToDevice));
    HJG_HIP(hipMemcpy(ab + o_fa, fa.data(), P * sizeof(FinalizeArgs), hipMemcpyHostToDevice));
    HJG_HIP(hipMemcpy(ab + o_ia, ia.data(), P * sizeof(InitArgs), hipMemcpyHostToDevice));
    HJG_HIP(hipMemcpy(ab + o_ra, ra.data(), P * sizeof(ReduceArgs), hipMemcpyHostToDevice));
    const SweepArgs* d_sa = (const SweepArgs*)(ab + o_sa);
    const FinalizeArgs* d_fa = (const FinalizeArgs*)(ab + o_fa);
    const InitArgs* d_ia = (const InitArgs*)(ab + o_ia);
    const ReduceArgs* d_ra = (const ReduceArgs*)(ab + o_ra);

    // ---- work items: init and finalize per register bucket, sweeps per
    //      specialisation, heaviest items first; reduce lists per level
    std::vector<int> items;   // int4 / int2 / int records, packed as ints
    struct Launch {
      int kind;     // 0 init, 1 sweep, 2 finalize, 3 reduce
      int rep;      // representative problem (specialisation)
      int64_t off;  // int offset in items
      int count;
      int level;
    };
    std::vector<Launch> launches;
    auto bucket_of = [&](int p) { return n_bucket(probs[p].n); };
    auto add_q_items = [&](int kind, int level) {
      std::map<int, std::vector<int>> byb;
      for (int p = 0; p < P; ++p)
        if (kind == 0 || Ks[p] > level) byb[bucket_of(p)].push_back(p);
      for (auto& kv : byb) {
        while (items.size() % 2) items.push_back(0);   // int2 records: 8-byte aligned
        const int64_t o = (int64_t)items.size();
        int cnt = 0;
        for (int p : kv.second)
          for (int64_t b = 0; b < pl[p].qb256; ++b, ++cnt) {
            items.push_back(p);
            items.push_back((int)b);
          }
        launches.push_back(Launch{kind, kv.second[0], o, cnt, level});
      }
    };
    add_q_items(0, 0);
    // One chain per kernel specialisation: its problems' levels in order
    // (sweep, finalize, reduce), independent of the other chains, so the
    // chains run as parallel graph branches without a barrier per level.
    std::map<SpecKey, std::vector<int>> groups;
    for (int p = 0; p < P; ++p) {
      const hjg_problem& pr = probs[p];
      const SpecKey sk{pr.datum, n_bucket(pr.n),
                       (pr.datum == HJG_L_MIN_PAIR_DISKS || pr.datum == HJG_L_CAPTURE) ? pr.n / 3 : 0, pl[p].mfma,
                       pl[p].bf16};
      groups[sk].push_back(p);
    }
    struct Chain {
      size_t first, last;   // launches [first, last)
      double cost;
    };
    std::vector<Chain> chains;
    for (auto& kv : groups) {
      const std::vector<int>& G = kv.second;
      Chain ch{launches.size(), 0, 0.0};
      int Kg = 0;
      for (int p : G) Kg = std::max(Kg, (int)Ks[p]);
      for (int k = 0; k < Kg; ++k) {
        struct It { int p, qb, sp; double cost; };
        std::vector<It> its;
        std::vector<int> live;
        for (int p : G) {
          if (Ks[p] <= k) continue;
          live.push_back(p);
          for (int64_t qb = 0; qb < pl[p].qb_sweep; ++qb)
            for (int sp = 0; sp < pl[p].splits; ++sp) {
              const int samples = std::min<int64_t>(pl[p].ns, (int64_t)Ns[p] - (int64_t)sp * pl[p].ns);
              its.push_back(It{p, (int)qb, sp, (double)samples * (probs[p].n + 10)});
            }
        }
        std::stable_sort(its.begin(), its.end(), [](const It& x, const It& y) { return x.cost > y.cost; });
        while (items.size() % 4) items.push_back(0);     // int4 records: 16-byte aligned
        int64_t o = (int64_t)items.size();
        for (const It& it : its) {
          items.push_back(it.p);
          items.push_back(it.qb);
          items.push_back(it.sp);
          items.push_back(0);
          ch.cost += it.cost;
        }
        launches.push_back(Launch{1, live[0], o, (int)its.size(), k});
        // finalize: (problem, 256-state block) records; one register bucket per chain
        while (items.size() % 2) items.push_back(0);     // int2 records: 8-byte aligned
        o = (int64_t)items.size();
        int cnt = 0;
        for (int p : live)
          for (int64_t b = 0; b < pl[p].qb256; ++b, ++cnt) {
            items.push_back(p);
            items.push_back((int)b);
          }
        launches.push_back(Launch{2, live[0], o, cnt, k});
        o = (int64_t)items.size();
        for (int p : live) items.push_back(p);
        launches.push_back(Launch{3, 0, o, (int)live.size(), k});
      }
      ch.last = launches.size();
      chains.push_back(ch);
    }
    // one work-queue head per sweep launch, after the item records
    int n_sweeps = 0;
    for (const Launch& L : launches) n_sweeps += L.kind == 1;
    while (items.size() % 4) items.push_back(0);
    const int64_t o_ctr = (int64_t)items.size();
    items.resize(items.size() + std::max(n_sweeps, 1), 0);
    if ((rc = ensure(ctx, B.items, std::max<size_t>(items.size(), 4) * sizeof(int)))) return rc;
    HJG_HIP(hipMemcpy(B.items.p, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice));
    const int* d_items = (const int*)B.items.p;
    int* d_ctr = (int*)B.items.p + o_ctr;
    const bool persistent = (mode & 1) != 0;

    // ---- common tables (and their column means), generated once per plan
    for (int p = 0; p < P; ++p) {
      const hjg_problem& pr = probs[p];
      const uint32_t k0 = (uint32_t)(pr.seed & 0xFFFFFFFFu), k1 = (uint32_t)(pr.seed >> 32);
      HJG_HIP(launch_table(pr.n, pl[p].tstride, pl[p].tstride, k0, k1, make_tag(pr.problem_id, 0, 0), pl[p].bf16,
                           at(pl[p].o_tab), s));
      if (pr.grad_cv)
        HJG_HIP(launch_zbar(pr.n, Ns[p], pl[p].tstride, pl[p].bf16, at(pl[p].o_tab), (double*)at(pl[p].o_zb), s));
      if (pl[p].o_zd >= 0)
        HJG_HIP(launch_pair_coords(pr.n / 3, Ns[p], pl[p].tstride, at(pl[p].o_tab), pair_coord_stride(pr.n / 3),
                                   (float*)at(pl[p].o_zd), s));
    }
    HJG_HIP(hipStreamSynchronize(s));

    // ---- record the whole uneven multi-problem Picard loop
    const bool concurrent = (mode & 2) != 0;
    if (concurrent && (rc = ensure_side(ctx))) return rc;
    HJG_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = persistent ? launch_fill_ints(d_ctr, n_sweeps, 0, ctx->cap) : hipSuccess;
    // sweep launch i uses work-queue head d_ctr[i], in launch-list order
    std::vector<int> qhead(launches.size(), 0);
    for (size_t li = 0, i = 0; li < launches.size(); ++li)
      if (launches[li].kind == 1) qhead[li] = (int)i++;
    auto record = [&](size_t li, hipStream_t st) -> hipError_t {
      const Launch& L = launches[li];
      if (L.kind == 0) {
        ItemBatch<InitArgs> b{d_ia, (const int2*)(d_items + L.off), L.count};
        return launch_init(ia[L.rep], st, &b);
      }
      if (L.kind == 1) {
        SweepBatch b{d_sa, (const int4*)(d_items + L.off), L.count, persistent ? d_ctr + qhead[li] : nullptr};
        return launch_sweep(sa[L.rep], 0, pl[L.rep].bf16, st, &b);
      }
      if (L.kind == 2) {
        ItemBatch<FinalizeArgs> b{d_fa, (const int2*)(d_items + L.off), L.count};
        return launch_finalize(fa[L.rep], st, &b);
      }
      return launch_reduce_batched(d_ra, d_items + L.off, L.count, L.level, st);
    };
    const size_t n_init = chains.empty() ? launches.size() : chains[0].first;
    for (size_t li = 0; li < n_init && e == hipSuccess; ++li) e = record(li, ctx->cap);
    if (concurrent && chains.size() > 1) {
      // chains onto the side streams, heaviest first to the least loaded
      // stream; join back at the end
      const int ns = (int)std::min<size_t>(chains.size(), hjg_ctx::kSide);
      std::vector<size_t> order(chains.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(),
                       [&](size_t a, size_t b) { return chains[a].cost > chains[b].cost; });
      std::vector<double> load(ns, 0.0);
      std::vector<std::vector<size_t>> lane(ns);
      for (size_t c : order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[j] += chains[c].cost;
        lane[j].push_back(c);
      }
      if (e == hipSuccess) e = hipEventRecord(ctx->fork_ev, ctx->cap);
      for (int j = 0; j < ns && e == hipSuccess; ++j) e = hipStreamWaitEvent(ctx->side[j], ctx->fork_ev, 0);
      for (int j = 0; j < ns && e == hipSuccess; ++j)
        for (size_t c : lane[j])
          for (size_t li = chains[c].first; li < chains[c].last && e == hipSuccess; ++li) e = record(li, ctx->side[j]);
      for (int j = 0; j < ns && e == hipSuccess; ++j) {
        e = hipEventRecord(ctx->join_ev[j], ctx->side[j]);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->cap, ctx->join_ev[j], 0);
      }
    } else {
      for (size_t li = n_init; li < launches.size() && e == hipSuccess; ++li) e = record(li, ctx->cap);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(HJG_EHIP, std::string("batched graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(HJG_EHIP, std::string("batched graph instantiate: ") + hipGetErrorString(e3));
    }
    B.graph = graph;
    B.exec = exec;
    B.key = key;
  }
  HJG_HIP(hipGraphLaunch(B.exec, s));
  // the next call that re-plans waits for this replay before it rewrites the
  // workspace, argument records and work items the replay reads
  HJG_HIP(hipEventRecord(B.replay_ev, s));
  if (resid_hist || iters) {
    std::vector<double> r;
    int64_t bad_states = 0;
    int first_bad = -1;
    for (int p = 0; p < P; ++p) {
      r.assign(B.K[p], 0.0);
      int ctrl[3] = {0, 0, 0};
      HJG_HIP(hipMemcpyAsync(r.data(), (char*)B.ws.p + B.resid_off[p], B.K[p] * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      HJG_HIP(hipMemcpyAsync(ctrl, (char*)B.ws.p + B.ctrl_off[p], 3 * sizeof(int), hipMemcpyDeviceToHost, s));
      HJG_HIP(hipStreamSynchronize(s));
      if (resid_hist)
        for (int k = 0; k < Kmax; ++k) resid_hist[(int64_t)p * Kmax + k] = k < B.K[p] ? r[k] : 0.0;
      if (iters) iters[p] = ctrl[1];
      if (ctrl[2] && first_bad < 0) first_bad = p;
      bad_states += ctrl[2];
    }
    if (bad_states)
      return fail(HJG_ENONFINITE, std::to_string(bad_states) + " states have a non-finite value or gradient "
                                  "(first in problem " + std::to_string(first_bad) + ")");
  }
  return HJG_OK;
}

// ===================================================================== flock
extern "C" int hjg_knn_grid(hjg_ctx* ctx, int64_t M, const float* pos, const float* box_lo, const float* box_hi,
                            float cell, int32_t k, int32_t* idx, float* nbr_pos, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_knn_grid");
  g_err.clear();
  if (!ctx) return fail(HJG_EINVAL, "NULL context");
  if (!pos || !box_lo || !box_hi) return fail(HJG_EINVAL, "pos, box_lo and box_hi are required");
  if (k < 1 || k > kMaxKnn) return fail(HJG_EINVAL, "k must be in 1..8");
  if (M < k + 1) return fail(HJG_EINVAL, "need more than k agents");
  if (M > INT32_MAX) return fail(HJG_EINVAL, "at most 2^31 - 1 agents");
  if (!(std::isfinite(cell) && cell > 0.f)) return fail(HJG_EINVAL, "cell must be finite and > 0");
  GridGeom gg{};
  int64_t cells = 1;
  for (int d = 0; d < 3; ++d) {
    if (!(std::isfinite(box_lo[d]) && std::isfinite(box_hi[d]) && box_hi[d] >= box_lo[d]))
      return fail(HJG_EINVAL, "box must be finite with hi >= lo");
    const double gd = std::ceil(((double)box_hi[d] - box_lo[d]) / cell);
    if (gd > (double)(1 << 20)) return fail(HJG_EINVAL, "more than 2^20 cells along one axis");
    gg.g[d] = std::max(1, (int)gd);
    gg.lo[d] = box_lo[d];
    cells *= gg.g[d];
  }
  if (cells >= kMaxGridCells) return fail(HJG_EINVAL, "2^26 or more grid cells; use a larger cell");
  gg.h = cell;
  gg.inv_h = 1.f / cell;
  if (!idx && !nbr_pos) return HJG_OK;
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  int rc;
  const int64_t nb = (cells + 1 + 4095) / 4096;
  if ((rc = ensure(ctx, ctx->g_cell, M * sizeof(int))) || (rc = ensure(ctx, ctx->g_rank, M * sizeof(int))) ||
      (rc = ensure(ctx, ctx->g_start, (cells + 1) * sizeof(int))) || (rc = ensure(ctx, ctx->g_bsum, nb * sizeof(int))) ||
      (rc = ensure(ctx, ctx->g_sorted, M * sizeof(float4))) || (rc = ensure(ctx, ctx->ctrl, kCtrlWords * sizeof(int))))
    return rc;
  // positions must be finite: the cell of a NaN is not defined
  int* flag = (int*)ctx->ctrl.p + 3;
  HJG_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  HJG_HIP(launch_finite_check(pos, 3 * M, flag, s));
  int host = 0;
  HJG_HIP(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HJG_HIP(hipStreamSynchronize(s));
  if (host) return fail(HJG_ENONFINITE, "non-finite agent position");
  HJG_HIP(launch_grid_build(pos, M, gg, (int*)ctx->g_cell.p, (int*)ctx->g_rank.p, (int*)ctx->g_start.p,
                            (int*)ctx->g_bsum.p, (float4*)ctx->g_sorted.p, s));
  HJG_HIP(launch_knn((const float4*)ctx->g_sorted.p, (const int*)ctx->g_start.p, pos, M, gg, k, idx, nbr_pos, s));
  return HJG_OK;
}

// ===================================================================== tuning
namespace {
// Scratch of the tuning runs, released on every return path.
struct TuneScratch {
  void* v = nullptr;
  void* g = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneScratch() {
    if (v) (void)hipFree(v);
    if (g) (void)hipFree(g);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};
}  // namespace

extern "C" int hjg_autotune_sweep(hjg_ctx* ctx, const hjg_problem* p, int64_t Q, const float* x, double t, int32_t N,
                                  const float* c, const float* theta, int32_t* best_blocks, double* best_ms,
                                  void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_autotune_sweep");
  g_err.clear();
  int rc = check_common(ctx, p, Q, t, N, 0);
  if (rc) return rc;
  if (Q < 1 || !x || !c || !best_blocks || !best_ms) return fail(HJG_EINVAL, "NULL argument or Q < 1");
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  TuneScratch sc;
  if (hipMalloc(&sc.v, Q * sizeof(float)) != hipSuccess || hipMalloc(&sc.g, (size_t)Q * p->n * sizeof(float)) != hipSuccess)
    return fail(HJG_ENOMEM, "autotuner scratch allocation failed");
  float* v = (float*)sc.v;
  float* g = (float*)sc.g;
  HJG_HIP(hipEventCreate(&sc.e0));
  HJG_HIP(hipEventCreate(&sc.e1));
  hipEvent_t e0 = sc.e0, e1 = sc.e1;
  const std::string key = sweep_key(p, Q, N);
  const int candidates[] = {512, 1024, 2048, 4096, 8192, 16384};
  double best = 1e300;
  int choice = 2048;
  for (int cand : candidates) {
    ctx->tuning[key] = cand;
    float total = 0.f;
    for (int rep = 0; rep < 4 && rc == HJG_OK; ++rep) {
      if (rep == 1) HJG_HIP(hipEventRecord(e0, s));
      rc = hjg_value_grad(ctx, p, Q, x, t, N, 0, 0, c, theta, v, g, nullptr, 0, hip_stream);
    }
    if (rc) break;
    HJG_HIP(hipEventRecord(e1, s));
    HJG_HIP(hipEventSynchronize(e1));
    HJG_HIP(hipEventElapsedTime(&total, e0, e1));
    if (total / 3.0 < best) {
      best = total / 3.0;
      choice = cand;
    }
  }
  if (rc) {
    ctx->tuning.erase(key);
    return rc;
  }
  ctx->tuning[key] = choice;
  *best_blocks = choice;
  *best_ms = best;
  return HJG_OK;
}

extern "C" int hjg_autotune_batched(hjg_ctx* ctx, int32_t P, const hjg_problem* probs, const int64_t* q_off,
                                    const int32_t* Ns, const int32_t* Ks, const double* ts, double tol,
                                    const float* x_all, float* v_all, float* grad_all, int32_t* best_split,
                                    double* best_ms, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_autotune_batched");
  g_err.clear();
  if (!ctx || !best_split || !best_ms) return fail(HJG_EINVAL, "NULL argument");
  HJG_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  TuneScratch sc;
  HJG_HIP(hipEventCreate(&sc.e0));
  HJG_HIP(hipEventCreate(&sc.e1));
  hipEvent_t e0 = sc.e0, e1 = sc.e1;
  const int candidates[] = {2048, 4096, 8192, 16384, 32768, 65536};
  double best = 1e300;
  int choice = 16384, rc = HJG_OK;
  for (int cand : candidates) {
    ctx->tuning["batch"] = cand;
    // first call records the plan, the second is timed
    rc = hjg_picard_sweep_batched(ctx, P, probs, q_off, Ns, Ks, ts, tol, x_all, v_all, grad_all, nullptr, nullptr,
                                  hip_stream);
    if (rc) break;
    HJG_HIP(hipEventRecord(e0, s));
    rc = hjg_picard_sweep_batched(ctx, P, probs, q_off, Ns, Ks, ts, tol, x_all, v_all, grad_all, nullptr, nullptr,
                                  hip_stream);
    if (rc) break;
    HJG_HIP(hipEventRecord(e1, s));
    HJG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HJG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      choice = cand;
    }
  }
  if (rc) {
    ctx->tuning.erase("batch");
    return rc;
  }
  ctx->tuning["batch"] = choice;
  // then the launch mode at that split (the default mode was timed above)
  const int mode0 = batched_mode(ctx);
  int mode_choice = mode0;
  for (int mode = 0; mode < 4 && rc == HJG_OK; ++mode) {
    if (mode == mode0) continue;
    ctx->tuning["batch_mode"] = mode + 1;
    if (batched_mode(ctx) != mode) continue;       // an environment override pins this bit
    rc = hjg_picard_sweep_batched(ctx, P, probs, q_off, Ns, Ks, ts, tol, x_all, v_all, grad_all, nullptr, nullptr,
                                  hip_stream);
    if (rc) break;
    HJG_HIP(hipEventRecord(e0, s));
    rc = hjg_picard_sweep_batched(ctx, P, probs, q_off, Ns, Ks, ts, tol, x_all, v_all, grad_all, nullptr, nullptr,
                                  hip_stream);
    if (rc) break;
    HJG_HIP(hipEventRecord(e1, s));
    HJG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HJG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      mode_choice = mode;
    }
  }
  ctx->tuning["batch_mode"] = mode_choice + 1;
  if (rc) return rc;
  *best_split = choice;
  *best_ms = best;
  return HJG_OK;
}

extern "C" int hjg_tuning_save(const hjg_ctx* ctx, const char* path) {
  g_err.clear();
  if (!ctx || !path) return fail(HJG_EINVAL, "NULL argument");
  std::ofstream f(path);
  if (!f) return fail(HJG_EINVAL, std::string("cannot write ") + path);
  f << "hjg-tuning gfx950 1\n";
  for (const auto& kv : ctx->tuning) f << kv.first << " = " << kv.second << "\n";
  return f ? HJG_OK : fail(HJG_EINVAL, std::string("write failed: ") + path);
}

extern "C" int hjg_tuning_load(hjg_ctx* ctx, const char* path) {
  g_err.clear();
  if (!ctx || !path) return fail(HJG_EINVAL, "NULL argument");
  std::ifstream f(path);
  if (!f) return fail(HJG_EINVAL, std::string("cannot read ") + path);
  std::string line;
  if (!std::getline(f, line) || line.rfind("hjg-tuning gfx950", 0) != 0)
    return fail(HJG_EINVAL, "not a gfx950 tuning file");
  std::map<std::string, int> table;
  while (std::getline(f, line)) {
    const size_t eq = line.rfind(" = ");
    if (line.empty()) continue;
    if (eq == std::string::npos) return fail(HJG_EINVAL, "malformed tuning line: " + line);
    const int v = std::atoi(line.c_str() + eq + 3);
    if (v < 1) return fail(HJG_EINVAL, "malformed tuning value: " + line);
    table[line.substr(0, eq)] = v;
  }
  ctx->tuning = table;
  return HJG_OK;
}
