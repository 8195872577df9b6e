// Surrogate network (x, t) -> (v, Dv): parameters, forward and backward on the
// matrix cores, AdamW training with a native data loader (per-epoch
// permutation), prediction, and the surrogate-accelerated sweep with
// plain Monte-Carlo fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hjg.h"
#include "internal.h"
#include "kernels.h"
#include "mlp.h"
#include "mlp_fused.h"

using namespace hjg;

namespace {

int fail(int code, const std::string& msg) { return hjg_internal_fail(code, msg.c_str()); }

#define SG_HIP(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(HJG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int round32(int v) { return (v + 31) / 32 * 32; }

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

int grow(Buf& b, size_t bytes) {
  if (bytes <= b.bytes) return HJG_OK;
  SG_HIP(hipDeviceSynchronize());
  if (b.p) SG_HIP(hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  if (hipMalloc(&b.p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HJG_ENOMEM, "surrogate workspace allocation failed");
  }
  b.bytes = std::max<size_t>(bytes, 256);
  return HJG_OK;
}

// splitmix64: seeds the host-side permutation and the initial weights
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-53; }

}  // namespace

struct hjg_surrogate {
  hjg_ctx* ctx = nullptr;
  int device = 0;
  int n = 0, width = 0, depth = 0;
  int nin = 0, nout = 0, in_p = 0, out_p = 0;
  int L = 0;                        // layers = depth + 1
  std::vector<int> fin, fout;       // padded fan-in / fan-out per layer
  std::vector<int> tin, tout;       // true fan-in / fan-out per layer
  std::vector<int64_t> woff, boff;  // offsets into the padded flat buffers
  int64_t P = 0;                    // padded parameter count
  Buf w, g, m, v;                   // float32 master weights, gradients, Adam moments
  std::vector<Buf> Wb, WbT;         // bfloat16 copies per layer
  Buf norm;                         // float32 [4][nin]: in mean, in std, out mean, out std
  Buf lw;                           // loss weights [out_p]
  int64_t step = 0;
  // batch workspace
  int64_t cap = 0;
  Buf X0, X0T, Y, T, dY, dYT, part, bl, acc, perm;
  Buf ctr;                          // training step counters (device)
  std::vector<Buf> Z, X, XT;
  Buf dZ[2], dZT[2];
  std::vector<Buf> dZTl;            // fused step: transposed errors of each hidden layer [width][B]
  Buf Xp, Tp, sched;                // fused step: the epoch's permuted training set; per-step schedule
  // training set and sweep workspace
  Buf Xall, Tall, sv, sg, tq, flags, bcount, total, index, xfb, vfb, gfb;
  // time-marching step workspace
  Buf mt_table, mt_zbar, mt_c, mt_th, mt_vprev, mt_pm, mt_pS, mt_pS2, mt_pG, mt_block, mt_resid, mt_ctrl;
};

namespace {

int ensure_batch(hjg_surrogate* s, int64_t rows, bool train) {
  int rc;
  if (rows <= s->cap && (!train || s->dY.bytes >= (size_t)rows * s->out_p * 2)) return HJG_OK;
  const int64_t r = std::max<int64_t>(rows, s->cap);
  if ((rc = grow(s->X0, r * s->in_p * 2))) return rc;
  if ((rc = grow(s->Y, r * s->out_p * 4))) return rc;
  s->Z.resize(s->depth);
  s->X.resize(s->depth);
  s->XT.resize(s->depth);
  for (int l = 0; l < s->depth; ++l)
    if ((rc = grow(s->X[l], r * s->width * 2))) return rc;
  if (train) {
    if ((rc = grow(s->X0T, r * s->in_p * 2))) return rc;
    if ((rc = grow(s->T, r * s->out_p * 4))) return rc;
    if ((rc = grow(s->dY, r * s->out_p * 2))) return rc;
    if ((rc = grow(s->dYT, r * s->out_p * 2))) return rc;
    for (int l = 0; l < s->depth; ++l) {
      if ((rc = grow(s->Z[l], r * s->width * 4))) return rc;
      if ((rc = grow(s->XT[l], r * s->width * 2))) return rc;
    }
    for (int i = 0; i < 2; ++i) {
      if ((rc = grow(s->dZ[i], r * s->width * 2))) return rc;
      if ((rc = grow(s->dZT[i], r * s->width * 2))) return rc;
    }
    s->dZTl.resize(s->depth);
    for (int l = 0; l < s->depth; ++l)
      if ((rc = grow(s->dZTl[l], r * s->width * 2))) return rc;
    if ((rc = grow(s->bl, (r * s->out_p / 256 + 2) * 8))) return rc;
    if ((rc = grow(s->acc, 64))) return rc;
  }
  s->cap = r;
  return HJG_OK;
}

int refresh_bf16(hjg_surrogate* s, hipStream_t st) {
  for (int l = 0; l < s->L; ++l)
    SG_HIP(launch_to_bf16((const float*)s->w.p + s->woff[l], s->fout[l], s->fin[l], (__bf16*)s->Wb[l].p,
                          (__bf16*)s->WbT[l].p, st));
  return HJG_OK;
}

const float* nrm(const hjg_surrogate* s, int which) { return (const float*)s->norm.p + which * s->nin; }

// Forward pass over `rows` rows of X0.  With `train`, also keeps the
// pre-activations and the transposed activations for the backward pass.
int forward(hjg_surrogate* s, int64_t rows, bool train, hipStream_t st) {
  const __bf16* h = (const __bf16*)s->X0.p;
  int ldh = s->in_p;
  for (int l = 0; l < s->depth; ++l) {
    GemmArgs a{};
    a.A = h;
    a.lda = ldh;
    a.B = (const __bf16*)s->Wb[l].p;
    a.ldb = s->fin[l];
    a.M = (int)rows;
    a.N = s->fout[l];
    a.K = s->fin[l];
    a.bias = (const float*)s->w.p + s->boff[l];
    a.outf = train ? (float*)s->Z[l].p : nullptr;
    a.ldo = s->width;
    a.outb = (__bf16*)s->X[l].p;
    a.ldob = s->width;
    a.outbT = train ? (__bf16*)s->XT[l].p : nullptr;
    a.ldobT = (int)rows;
    SG_HIP(launch_gemm(EPI_FWD_HIDDEN, a, 1, st));
    h = (const __bf16*)s->X[l].p;
    ldh = s->width;
  }
  GemmArgs a{};
  a.A = h;
  a.lda = ldh;
  a.B = (const __bf16*)s->Wb[s->depth].p;
  a.ldb = s->width;
  a.M = (int)rows;
  a.N = s->out_p;
  a.K = s->width;
  a.bias = (const float*)s->w.p + s->boff[s->depth];
  a.outf = (float*)s->Y.p;
  a.ldo = s->out_p;
  SG_HIP(launch_gemm(EPI_FWD_OUT, a, 1, st));
  return HJG_OK;
}

// Loss (added to s->acc[0]) and gradients of all parameters into s->g for a
// batch already forwarded with train = true, targets in s->T.
int backward(hjg_surrogate* s, int64_t rows, hipStream_t st) {
  int rc;
  const int B = (int)rows;
  int nb = 0;
  SG_HIP(launch_mse_loss((const float*)s->Y.p, (const float*)s->T.p, (const float*)s->lw.p, B, s->nout, s->out_p,
                         (__bf16*)s->dY.p, (__bf16*)s->dYT.p, (double*)s->bl.p, &nb, st));
  SG_HIP(launch_accumulate((const double*)s->bl.p, nb, (double*)s->acc.p, st));
  const int kps = 256;   // batch rows per weight-gradient split (one LDS round each)
  const int splits = (B + kps - 1) / kps;
  // weight-gradient partials [splits][M][N], then the bias partials [splits][M]
  if ((rc = grow(s->part, (size_t)splits * s->width * std::max(s->width, s->in_p) * 4 +
                              (size_t)splits * s->out_p * s->width * 4 +
                              (size_t)splits * std::max(s->width, s->out_p) * 4)))
    return rc;
  float* g = (float*)s->g.p;
  // output layer
  {
    const int l = s->depth;
    GemmArgs a{};
    a.A = (const __bf16*)s->dYT.p;
    a.lda = B;
    a.B = (const __bf16*)s->XT[l - 1].p;
    a.ldb = B;
    a.M = s->out_p;
    a.N = s->width;
    a.K = B;
    a.k_per_split = kps;
    a.outf = (float*)s->part.p;
    a.ldo = s->width;
    a.pbias = (float*)s->part.p + (size_t)splits * s->out_p * s->width;
    SG_HIP(launch_gemm(EPI_DW, a, splits, st));
    SG_HIP(launch_sum_splits((const float*)s->part.p, splits, s->out_p, s->width, s->width, g + s->woff[l], s->width,
                             a.pbias, g + s->boff[l], st));
    GemmArgs d{};
    d.A = (const __bf16*)s->dY.p;
    d.lda = s->out_p;
    d.B = (const __bf16*)s->WbT[l].p;
    d.ldb = s->out_p;
    d.M = B;
    d.N = s->width;
    d.K = s->out_p;
    d.outb = (__bf16*)s->dZ[0].p;
    d.ldob = s->width;
    d.outbT = (__bf16*)s->dZT[0].p;
    d.ldobT = B;
    d.zprev = (const float*)s->Z[l - 1].p;
    d.ldz = s->width;
    SG_HIP(launch_gemm(EPI_BWD_DX, d, 1, st));
  }
  int cur = 0;
  for (int l = s->depth - 1; l >= 0; --l) {
    const __bf16* inT = l == 0 ? (const __bf16*)s->X0T.p : (const __bf16*)s->XT[l - 1].p;
    GemmArgs a{};
    a.A = (const __bf16*)s->dZT[cur].p;
    a.lda = B;
    a.B = inT;
    a.ldb = B;
    a.M = s->width;
    a.N = s->fin[l];
    a.K = B;
    a.k_per_split = kps;
    a.outf = (float*)s->part.p;
    a.ldo = s->fin[l];
    a.pbias = (float*)s->part.p + (size_t)splits * s->width * s->fin[l];
    SG_HIP(launch_gemm(EPI_DW, a, splits, st));
    SG_HIP(launch_sum_splits((const float*)s->part.p, splits, s->width, s->fin[l], s->fin[l], g + s->woff[l],
                             s->fin[l], a.pbias, g + s->boff[l], st));
    if (l > 0) {
      GemmArgs d{};
      d.A = (const __bf16*)s->dZ[cur].p;
      d.lda = s->width;
      d.B = (const __bf16*)s->WbT[l].p;
      d.ldb = s->width;
      d.M = B;
      d.N = s->width;
      d.K = s->width;
      d.outb = (__bf16*)s->dZ[1 - cur].p;
      d.ldob = s->width;
      d.outbT = (__bf16*)s->dZT[1 - cur].p;
      d.ldobT = B;
      d.zprev = (const float*)s->Z[l - 1].p;
      d.ldz = s->width;
      SG_HIP(launch_gemm(EPI_BWD_DX, d, 1, st));
      cur = 1 - cur;
    }
  }
  return HJG_OK;
}

// The fused training step (two launches: rows, then weight gradients with
// AdamW) serves the network shapes and batch sizes its kernels are
// instantiated for; HJG_MLP_FUSED=0 selects the layer-by-layer launches
// instead.
bool fused_ok(const hjg_surrogate* s, int64_t B) {
  const char* e = std::getenv("HJG_MLP_FUSED");
  if (e && e[0] == '0') return false;
  return fused_rows_supported(s->width, s->in_p, s->out_p, s->depth) && B <= INT32_MAX &&
         fused_weights_supported((int)B);
}

FusedRowsArgs fused_rows_args(hjg_surrogate* s, int B, const __bf16* X, const float* T, int64_t row0) {
  FusedRowsArgs a{};
  const float* w = (const float*)s->w.p;
  int k = 0;
  for (int l = 0; l <= s->depth; ++l) {
    FusedPhase& P = a.ph[k++];
    P.W = (const __bf16*)s->Wb[l].p;
    P.bias = w + s->boff[l];
    P.outT = l < s->depth ? (__bf16*)s->XT[l].p : (__bf16*)s->dYT.p;
  }
  for (int l = s->depth; l >= 1; --l) {
    FusedPhase& P = a.ph[k++];
    P.W = (const __bf16*)s->WbT[l].p;
    P.bias = nullptr;
    P.outT = (__bf16*)s->dZTl[l - 1].p;
  }
  a.X = X;
  a.T = T;
  a.row0 = row0;
  a.B = B;
  a.in_p = s->in_p;
  a.out_p = s->out_p;
  a.nout = s->nout;
  a.lw = (const float*)s->lw.p;
  a.X0T = (__bf16*)s->X0T.p;
  a.block_loss = (double*)s->bl.p;
  return a;
}

FusedWeightsArgs fused_weights_args(hjg_surrogate* s, int B) {
  FusedWeightsArgs a{};
  a.L = s->L;
  a.B = B;
  int tiles = 0;
  for (int l = 0; l < s->L; ++l) {
    FusedLayer& Y = a.layer[l];
    Y.A = l < s->depth ? (const __bf16*)s->dZTl[l].p : (const __bf16*)s->dYT.p;
    Y.Bm = l == 0 ? (const __bf16*)s->X0T.p : (const __bf16*)s->XT[l - 1].p;
    Y.fin = s->fin[l];
    Y.fout = s->fout[l];
    Y.woff = s->woff[l];
    Y.boff = s->boff[l];
    Y.Wb = (__bf16*)s->Wb[l].p;
    Y.WbT = (__bf16*)s->WbT[l].p;
    Y.tiles_n = s->fin[l] / 32;
    Y.first = tiles;
    tiles += (s->fout[l] / 32) * Y.tiles_n;
  }
  a.tiles = tiles;
  a.w = (float*)s->w.p;
  a.g = (float*)s->g.p;
  a.m = (float*)s->m.p;
  a.v = (float*)s->v.p;
  a.block_loss = (const double*)s->bl.p;
  a.nbl = B / kFusedRows;
  a.acc = (double*)s->acc.p;
  return a;
}

}  // namespace

extern "C" {

int hjg_surrogate_create(hjg_ctx* ctx, int32_t n, int32_t width, int32_t depth, uint64_t seed, hjg_surrogate** out) {
  if (!ctx || !out) return fail(HJG_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > 96) return fail(HJG_EINVAL, "n must be in [1, 96]");
  if (width < 32 || width > 1024 || width % 32) return fail(HJG_EINVAL, "width must be a multiple of 32 in [32, 1024]");
  if (depth < 1 || depth > 16) return fail(HJG_EINVAL, "depth must be in [1, 16]");
  int device = 0;
  SG_HIP(hipGetDevice(&device));
  auto* s = new hjg_surrogate();
  s->ctx = ctx;
  s->device = device;
  s->n = n;
  s->width = width;
  s->depth = depth;
  s->nin = s->nout = n + 1;
  s->in_p = round32(s->nin);
  s->out_p = round32(s->nout);
  s->L = depth + 1;
  int64_t off = 0;
  for (int l = 0; l < s->L; ++l) {
    s->fin.push_back(l == 0 ? s->in_p : width);
    s->fout.push_back(l == depth ? s->out_p : width);
    s->tin.push_back(l == 0 ? s->nin : width);
    s->tout.push_back(l == depth ? s->nout : width);
    s->woff.push_back(off);
    off += (int64_t)s->fin[l] * s->fout[l];
    s->boff.push_back(off);
    off += s->fout[l];
  }
  s->P = off;
  int rc = 0;
  auto cleanup = [&](int code) {
    hjg_surrogate_destroy(s);
    return code;
  };
  for (Buf* b : {&s->w, &s->g, &s->m, &s->v})
    if ((rc = grow(*b, s->P * 4))) return cleanup(rc);
  s->Wb.resize(s->L);
  s->WbT.resize(s->L);
  for (int l = 0; l < s->L; ++l) {
    if ((rc = grow(s->Wb[l], (size_t)s->fin[l] * s->fout[l] * 2))) return cleanup(rc);
    if ((rc = grow(s->WbT[l], (size_t)s->fin[l] * s->fout[l] * 2))) return cleanup(rc);
  }
  if ((rc = grow(s->norm, 4 * s->nin * 4))) return cleanup(rc);
  if ((rc = grow(s->lw, s->out_p * 4))) return cleanup(rc);
  // Uniform initial weights, He scale sqrt(6/fan_in) for the SiLU layers and
  // Glorot scale sqrt(6/(fan_in+fan_out)) for the linear output layer (zero
  // padding, zero biases); identity normalisation
  std::vector<float> hw(s->P, 0.f);
  uint64_t st = seed ^ 0x5DEECE66Dull;
  for (int l = 0; l < s->L; ++l) {
    const double lim = l < depth ? std::sqrt(6.0 / s->tin[l]) : std::sqrt(6.0 / (s->tin[l] + s->tout[l]));
    for (int o = 0; o < s->tout[l]; ++o)
      for (int i = 0; i < s->tin[l]; ++i)
        hw[s->woff[l] + (int64_t)o * s->fin[l] + i] = (float)((2.0 * uniform01(st) - 1.0) * lim);
  }
  std::vector<float> hn(4 * s->nin, 0.f);
  for (int i = 0; i < s->nin; ++i) hn[s->nin + i] = hn[3 * s->nin + i] = 1.f;
  if (hipMemcpy(s->w.p, hw.data(), s->P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->norm.p, hn.data(), hn.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s->m.p, 0, s->P * 4) != hipSuccess || hipMemset(s->v.p, 0, s->P * 4) != hipSuccess ||
      hipMemset(s->g.p, 0, s->P * 4) != hipSuccess)
    return cleanup(fail(HJG_EHIP, "surrogate initialisation copy failed"));
  if ((rc = refresh_bf16(s, nullptr))) return cleanup(rc);
  if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(HJG_EHIP, "surrogate initialisation failed"));
  *out = s;
  return HJG_OK;
}

void hjg_surrogate_destroy(hjg_surrogate* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  std::vector<Buf*> all = {&s->w, &s->g, &s->m, &s->v, &s->norm, &s->lw, &s->X0, &s->X0T, &s->Y, &s->T, &s->dY,
                           &s->dYT, &s->part, &s->bl, &s->acc, &s->perm, &s->ctr, &s->Xall, &s->Tall, &s->sv,
                           &s->sg,
                           &s->tq, &s->flags, &s->bcount, &s->total, &s->index, &s->xfb, &s->vfb, &s->gfb,
                           &s->dZ[0], &s->dZ[1], &s->dZT[0], &s->dZT[1], &s->Xp, &s->Tp, &s->sched,
                           &s->mt_table, &s->mt_zbar, &s->mt_c, &s->mt_th, &s->mt_vprev, &s->mt_pm, &s->mt_pS,
                           &s->mt_pS2, &s->mt_pG, &s->mt_block, &s->mt_resid, &s->mt_ctrl};
  for (auto& b : s->Wb) all.push_back(&b);
  for (auto& b : s->WbT) all.push_back(&b);
  for (auto& b : s->Z) all.push_back(&b);
  for (auto& b : s->X) all.push_back(&b);
  for (auto& b : s->XT) all.push_back(&b);
  for (auto& b : s->dZTl) all.push_back(&b);
  for (Buf* b : all)
    if (b->p) (void)hipFree(b->p);
  delete s;
}

int hjg_surrogate_param_count(const hjg_surrogate* s, int64_t* count) {
  if (!s || !count) return fail(HJG_EINVAL, "NULL argument");
  int64_t c = 0;
  for (int l = 0; l < s->L; ++l) c += (int64_t)s->tin[l] * s->tout[l] + s->tout[l];
  *count = c;
  return HJG_OK;
}

int hjg_surrogate_set_params(hjg_surrogate* s, const float* params, const float* norm) {
  if (!s || !params || !norm) return fail(HJG_EINVAL, "NULL argument");
  for (int i = 0; i < s->nin; ++i)
    if (!(norm[s->nin + i] > 0) || !(norm[3 * s->nin + i] > 0)) return fail(HJG_EINVAL, "std entries must be > 0");
  std::vector<float> hw(s->P, 0.f);
  int64_t k = 0;
  for (int l = 0; l < s->L; ++l) {
    for (int o = 0; o < s->tout[l]; ++o)
      for (int i = 0; i < s->tin[l]; ++i) hw[s->woff[l] + (int64_t)o * s->fin[l] + i] = params[k++];
    for (int o = 0; o < s->tout[l]; ++o) hw[s->boff[l] + o] = params[k++];
  }
  SG_HIP(hipMemcpy(s->w.p, hw.data(), s->P * 4, hipMemcpyHostToDevice));
  SG_HIP(hipMemcpy(s->norm.p, norm, 4 * s->nin * 4, hipMemcpyHostToDevice));
  SG_HIP(hipMemset(s->m.p, 0, s->P * 4));
  SG_HIP(hipMemset(s->v.p, 0, s->P * 4));
  s->step = 0;
  int rc = refresh_bf16(s, nullptr);
  if (rc) return rc;
  SG_HIP(hipDeviceSynchronize());
  return HJG_OK;
}

int hjg_surrogate_get_params(const hjg_surrogate* s, float* params, float* norm) {
  if (!s || !params) return fail(HJG_EINVAL, "NULL argument");
  SG_HIP(hipDeviceSynchronize());
  std::vector<float> hw(s->P);
  SG_HIP(hipMemcpy(hw.data(), s->w.p, s->P * 4, hipMemcpyDeviceToHost));
  int64_t k = 0;
  for (int l = 0; l < s->L; ++l) {
    for (int o = 0; o < s->tout[l]; ++o)
      for (int i = 0; i < s->tin[l]; ++i) params[k++] = hw[s->woff[l] + (int64_t)o * s->fin[l] + i];
    for (int o = 0; o < s->tout[l]; ++o) params[k++] = hw[s->boff[l] + o];
  }
  if (norm) SG_HIP(hipMemcpy(norm, s->norm.p, 4 * s->nin * 4, hipMemcpyDeviceToHost));
  return HJG_OK;
}

// File layout (little-endian): the 8 bytes "HJGSURR1", int32 n, width, depth,
// int32 0, int64 parameter count, float32 parameters (exchange format),
// float32 normalisation [4][n + 1].
int hjg_surrogate_save(const hjg_surrogate* s, const char* path) {
  if (!s || !path) return fail(HJG_EINVAL, "NULL argument");
  int64_t count = 0;
  int rc = hjg_surrogate_param_count(s, &count);
  if (rc) return rc;
  std::vector<float> params((size_t)count), norm((size_t)4 * s->nin);
  if ((rc = hjg_surrogate_get_params(s, params.data(), norm.data()))) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(HJG_EINVAL, std::string("cannot open ") + path + " for writing");
  const int32_t hdr[4] = {s->n, s->width, s->depth, 0};
  bool ok = std::fwrite("HJGSURR1", 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
            std::fwrite(&count, 8, 1, f) == 1 && std::fwrite(params.data(), 4, params.size(), f) == params.size() &&
            std::fwrite(norm.data(), 4, norm.size(), f) == norm.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(HJG_EINVAL, std::string("writing ") + path + " failed");
  return HJG_OK;
}

int hjg_surrogate_load(hjg_ctx* ctx, const char* path, hjg_surrogate** out) {
  if (!ctx || !path || !out) return fail(HJG_EINVAL, "NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(HJG_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[4];
  int64_t count = 0;
  auto bad = [&](const std::string& why) {
    std::fclose(f);
    return fail(HJG_EINVAL, std::string(path) + ": " + why);
  };
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "HJGSURR1", 8) != 0) return bad("not a surrogate file");
  if (std::fread(hdr, 4, 4, f) != 4 || std::fread(&count, 8, 1, f) != 1) return bad("truncated header");
  hjg_surrogate* s = nullptr;
  int rc = hjg_surrogate_create(ctx, hdr[0], hdr[1], hdr[2], 0, &s);
  if (rc) {
    std::fclose(f);
    return rc;
  }
  int64_t expect = 0;
  hjg_surrogate_param_count(s, &expect);
  std::vector<float> params, norm((size_t)4 * s->nin);
  bool ok = count == expect;
  if (ok) {
    params.resize((size_t)count);
    char extra;
    ok = std::fread(params.data(), 4, params.size(), f) == params.size() &&
         std::fread(norm.data(), 4, norm.size(), f) == norm.size() && std::fread(&extra, 1, 1, f) == 0;
  }
  std::fclose(f);
  if (!ok) {
    hjg_surrogate_destroy(s);
    return fail(HJG_EINVAL, std::string(path) + ": parameter count or size does not match the header");
  }
  if ((rc = hjg_surrogate_set_params(s, params.data(), norm.data()))) {
    hjg_surrogate_destroy(s);
    return rc;
  }
  *out = s;
  return HJG_OK;
}

int hjg_surrogate_predict(hjg_surrogate* s, int64_t Q, const float* x, const float* t, float* v, float* grad,
                          void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_surrogate_predict");
  if (!s) return fail(HJG_EINVAL, "surrogate is NULL");
  if (Q < 0) return fail(HJG_EINVAL, "Q must be >= 0");
  if (Q == 0) return HJG_OK;
  if (!x || !t || !v || !grad) return fail(HJG_EINVAL, "x, t, v and grad are required");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t chunk = 65536;
  int rc;
  if ((rc = ensure_batch(s, std::min(Q, chunk), false))) return rc;
  for (int64_t r0 = 0; r0 < Q; r0 += chunk) {
    const int64_t rows = std::min(chunk, Q - r0);
    SG_HIP(launch_prep_inputs(x + r0, Q, t + r0, s->n, rows, s->in_p, nrm(s, 0), nrm(s, 1), (__bf16*)s->X0.p,
                              nullptr, st));
    if ((rc = forward(s, rows, false, st))) return rc;
    SG_HIP(launch_post_outputs((const float*)s->Y.p, s->n, rows, s->out_p, nrm(s, 2), nrm(s, 3), v + r0, grad + r0,
                               Q, st));
  }
  return HJG_OK;
}

namespace {

int set_loss_weights(hjg_surrogate* s, double grad_weight, hipStream_t st) {
  std::vector<float> w(s->out_p, 0.f);
  w[0] = 1.f;
  for (int j = 1; j < s->nout; ++j) w[j] = (float)(grad_weight / s->n);
  SG_HIP(hipMemcpyAsync(s->lw.p, w.data(), w.size() * 4, hipMemcpyHostToDevice, st));
  SG_HIP(hipStreamSynchronize(st));
  return HJG_OK;
}

}  // namespace

int hjg_surrogate_loss_grad(hjg_surrogate* s, int64_t B, const float* x, const float* t, const float* v,
                            const float* grad, double grad_weight, double* loss, float* grads, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_surrogate_loss_grad");
  if (!s || !loss) return fail(HJG_EINVAL, "NULL argument");
  if (B < 32 || B % 32) return fail(HJG_EINVAL, "B must be a positive multiple of 32");
  if (!x || !t || !v || !grad) return fail(HJG_EINVAL, "x, t, v and grad are required");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc;
  if ((rc = ensure_batch(s, B, true))) return rc;
  if ((rc = set_loss_weights(s, grad_weight, st))) return rc;
  SG_HIP(launch_prep_inputs(x, B, t, s->n, B, s->in_p, nrm(s, 0), nrm(s, 1), (__bf16*)s->X0.p, (__bf16*)s->X0T.p,
                            st));
  SG_HIP(launch_prep_targets(v, grad, s->n, B, s->out_p, nrm(s, 2), nrm(s, 3), (float*)s->T.p, st));
  SG_HIP(hipMemsetAsync(s->acc.p, 0, 8, st));
  if (fused_ok(s, B)) {
    const FusedRowsArgs ra = fused_rows_args(s, (int)B, (const __bf16*)s->X0.p, (const float*)s->T.p, 0);
    SG_HIP(launch_fused_rows(ra, s->width, s->depth, st));
    FusedWeightsArgs wa = fused_weights_args(s, (int)B);
    wa.adam = 0;
    SG_HIP(launch_fused_weights(wa, st));
  } else {
    if ((rc = forward(s, B, true, st))) return rc;
    if ((rc = backward(s, B, st))) return rc;
  }
  double l = 0.0;
  SG_HIP(hipMemcpyAsync(&l, s->acc.p, 8, hipMemcpyDeviceToHost, st));
  SG_HIP(hipStreamSynchronize(st));
  *loss = l / (double)B;
  if (grads) {
    std::vector<float> hg(s->P);
    SG_HIP(hipMemcpy(hg.data(), s->g.p, s->P * 4, hipMemcpyDeviceToHost));
    int64_t k = 0;
    for (int l2 = 0; l2 < s->L; ++l2) {
      for (int o = 0; o < s->tout[l2]; ++o)
        for (int i = 0; i < s->tin[l2]; ++i) grads[k++] = hg[s->woff[l2] + (int64_t)o * s->fin[l2] + i];
      for (int o = 0; o < s->tout[l2]; ++o) grads[k++] = hg[s->boff[l2] + o];
    }
  }
  return HJG_OK;
}

int hjg_surrogate_train(hjg_surrogate* s, int64_t M, const float* x, const float* t, const float* v,
                        const float* grad, const hjg_train_cfg* cfg, double* loss_hist, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_surrogate_train");
  if (!s || !cfg) return fail(HJG_EINVAL, "NULL argument");
  if (!x || !t || !v || !grad) return fail(HJG_EINVAL, "x, t, v and grad are required");
  const int B = cfg->batch;
  if (B < 32 || B % 32 || B > (1 << 20)) return fail(HJG_EINVAL, "batch must be a multiple of 32 in [32, 2^20]");
  if (M < B) return fail(HJG_EINVAL, "need at least one full batch of training rows");
  if (cfg->epochs < 1 || !(cfg->lr > 0) || !(cfg->lr_min >= 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) ||
      !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0) || !(cfg->weight_decay >= 0))
    return fail(HJG_EINVAL, "invalid training configuration");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc;
  if ((rc = ensure_batch(s, B, true))) return rc;
  if ((rc = set_loss_weights(s, cfg->grad_weight, st))) return rc;
  // normalisation from the training data
  float* nm = (float*)s->norm.p;
  SG_HIP(launch_feature_stats(x, M, s->n, M, nm, nm + s->nin, st));
  SG_HIP(launch_feature_stats(t, M, 1, M, nm + s->n, nm + s->nin + s->n, st));
  SG_HIP(launch_feature_stats(v, M, 1, M, nm + 2 * s->nin, nm + 3 * s->nin, st));
  SG_HIP(launch_feature_stats(grad, M, s->n, M, nm + 2 * s->nin + 1, nm + 3 * s->nin + 1, st));
  // the whole normalised training set, inputs in bfloat16
  if ((rc = grow(s->Xall, (size_t)M * s->in_p * 2))) return rc;
  if ((rc = grow(s->Tall, (size_t)M * s->out_p * 4))) return rc;
  if ((rc = grow(s->perm, (size_t)M * 4))) return rc;
  SG_HIP(launch_prep_inputs(x, M, t, s->n, M, s->in_p, nrm(s, 0), nrm(s, 1), (__bf16*)s->Xall.p, nullptr, st));
  SG_HIP(launch_prep_targets(v, grad, s->n, M, s->out_p, nrm(s, 2), nrm(s, 3), (float*)s->Tall.p, st));
  const int64_t steps_per_epoch = M / B;
  const int64_t total = steps_per_epoch * cfg->epochs;
  if ((rc = grow(s->ctr, 3 * sizeof(int64_t)))) return rc;
  int64_t* ctr = (int64_t*)s->ctr.p;
  // One training step: batch gather, forward, backward, AdamW with the bf16
  // weight refresh.  The layer-by-layer step takes its batch, learning rate
  // and bias corrections from device counters that it advances; its first
  // step runs directly, the rest replay recorded graphs of one or G steps.
  if (s->L > kMaxLayers) return fail(HJG_EINVAL, "too many layers for the fused optimizer step");
  LayerTab tab{};
  tab.L = s->L;
  for (int l = 0; l < s->L; ++l) {
    tab.woff[l] = s->woff[l];
    tab.fin[l] = s->fin[l];
    tab.fout[l] = s->fout[l];
    tab.Wb[l] = (__bf16*)s->Wb[l].p;
    tab.WbT[l] = (__bf16*)s->WbT[l].p;
  }
  const bool fused = fused_ok(s, B);
  const char* ng = std::getenv("HJG_NO_GRAPH");       // 1: every step launched directly (for comparison)
  const bool use_graph = !(ng && ng[0] == '1');
  // The fused step takes fixed arguments: its rows of the epoch's permuted
  // training set and its entry of the epoch's schedule table (learning rate
  // and bias corrections formed on the host), so a whole epoch records as
  // one graph (up to kEpochGraphSteps steps; longer epochs launch directly).
  constexpr int64_t kEpochGraphSteps = 8192;
  FusedRowsArgs fra{};
  FusedWeightsArgs fwa{};
  std::vector<float> hsched;
  if (fused) {
    if ((rc = grow(s->Xp, (size_t)steps_per_epoch * B * s->in_p * 2)) ||
        (rc = grow(s->Tp, (size_t)steps_per_epoch * B * s->out_p * 4)) ||
        (rc = grow(s->sched, (size_t)steps_per_epoch * 3 * 4)))
      return rc;
    fra = fused_rows_args(s, B, (const __bf16*)s->Xp.p, (const float*)s->Tp.p, 0);
    fwa = fused_weights_args(s, B);
    fwa.adam = 1;
    fwa.b1 = (float)cfg->beta1;
    fwa.b2 = (float)cfg->beta2;
    fwa.eps = (float)cfg->eps;
    fwa.wd = (float)cfg->weight_decay;
    hsched.resize((size_t)steps_per_epoch * 3);
  }
  auto fused_step = [&](int64_t b, hipStream_t q) -> int {
    FusedRowsArgs ra = fra;
    ra.row0 = b * B;
    FusedWeightsArgs wa = fwa;
    wa.sched = (const float*)s->sched.p + 3 * b;
    SG_HIP(launch_fused_rows(ra, s->width, s->depth, q));
    SG_HIP(launch_fused_weights(wa, q));
    return HJG_OK;
  };
  auto train_step = [&](hipStream_t q) -> int {
    int r;
    SG_HIP(launch_gather((const __bf16*)s->Xall.p, (const float*)s->Tall.p, (const int*)s->perm.p, B, s->in_p,
                         s->out_p, ctr + 2, (__bf16*)s->X0.p, (__bf16*)s->X0T.p, (float*)s->T.p, q));
    if ((r = forward(s, B, true, q))) return r;
    if ((r = backward(s, B, q))) return r;
    SG_HIP(launch_adamw_sched((float*)s->w.p, (const float*)s->g.p, (float*)s->m.p, (float*)s->v.p, s->P, ctr,
                              cfg->lr, cfg->lr_min, total, (float)cfg->beta1, (float)cfg->beta2, (float)cfg->eps,
                              (float)cfg->weight_decay, &tab, q));
    SG_HIP(launch_advance_counters(ctr, q));
    return HJG_OK;
  };
  // Recorded graphs: the fused path's epoch (index 2); the layer-by-layer
  // path's one and G steps (indices 0, 1: the device counters move every step
  // on, so a graph of G steps replays G consecutive steps).
  const int64_t G = std::min<int64_t>(16, steps_per_epoch);
  hipStream_t cap = nullptr;
  hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  auto release = [&](int code) {
    for (int i = 0; i < 3; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
    if (cap) (void)hipStreamDestroy(cap);
    return code;
  };
  auto record = [&](int i) -> int {
    if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(HJG_EHIP, "training: graph capture could not start");
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(HJG_EHIP, "training: graph capture could not start");
    int r = HJG_OK;
    const int64_t steps = i == 2 ? steps_per_epoch : i == 1 ? G : 1;
    for (int64_t k = 0; k < steps && !r; ++k) r = i == 2 ? fused_step(k, cap) : train_step(cap);
    const hipError_t ec = hipStreamEndCapture(cap, &graph[i]);
    if (r) return r;
    if (ec != hipSuccess || hipGraphInstantiate(&exec[i], graph[i], nullptr, nullptr, 0) != hipSuccess)
      return fail(HJG_EHIP, "training: graph capture failed");
    return HJG_OK;
  };
  std::vector<int> perm(M);
  uint64_t seed = cfg->seed;
  for (int e = 0; e < cfg->epochs; ++e) {
    for (int64_t i = 0; i < M; ++i) perm[i] = (int)i;
    for (int64_t i = M - 1; i > 0; --i) {        // Fisher-Yates
      const int64_t j = (int64_t)(splitmix64(seed) % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    const int64_t c0[3] = {e * steps_per_epoch, s->step + e * steps_per_epoch, 0};
    if (hipMemcpyAsync(s->perm.p, perm.data(), (size_t)M * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ctr, c0, sizeof(c0), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(s->acc.p, 0, 8, st) != hipSuccess)
      return release(fail(HJG_EHIP, "training: upload of the epoch's order failed"));
    if (fused) {
      // cosine learning rate at global step k, bias corrections at optimizer step t
      for (int64_t b = 0; b < steps_per_epoch; ++b) {
        const double k = (double)(e * steps_per_epoch + b), t_opt = (double)(s->step + e * steps_per_epoch + b + 1);
        hsched[3 * b] = (float)(cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(M_PI * k / (double)total)));
        hsched[3 * b + 1] = (float)(1.0 - std::pow((double)(float)cfg->beta1, t_opt));
        hsched[3 * b + 2] = (float)(1.0 - std::pow((double)(float)cfg->beta2, t_opt));
      }
      if (hipMemcpyAsync(s->sched.p, hsched.data(), hsched.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
        return release(fail(HJG_EHIP, "training: upload of the epoch's schedule failed"));
      SG_HIP(launch_permute_rows((const __bf16*)s->Xall.p, (const float*)s->Tall.p, (const int*)s->perm.p,
                                 steps_per_epoch * B, s->in_p, s->out_p, (__bf16*)s->Xp.p, (float*)s->Tp.p, st));
      if (use_graph && steps_per_epoch <= kEpochGraphSteps) {
        if (!exec[2] && (rc = record(2))) return release(rc);
        if (hipGraphLaunch(exec[2], st) != hipSuccess) return release(fail(HJG_EHIP, "training: graph launch failed"));
      } else {
        for (int64_t b = 0; b < steps_per_epoch; ++b)
          if ((rc = fused_step(b, st))) return release(rc);
      }
    } else {
      for (int64_t b = 0; b < steps_per_epoch;) {
        if (!use_graph || (e == 0 && b == 0)) {
          if ((rc = train_step(st))) return release(rc);
          ++b;
          continue;
        }
        const int i = steps_per_epoch - b >= G ? 1 : 0;
        if (!exec[i] && (rc = record(i))) return release(rc);
        if (hipGraphLaunch(exec[i], st) != hipSuccess) return release(fail(HJG_EHIP, "training: graph launch failed"));
        b += i ? G : 1;
      }
    }
    double acc = 0.0;
    if (hipMemcpyAsync(&acc, s->acc.p, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)     // the host buffers are reused next epoch
      return release(fail(HJG_EHIP, "training: loss read-back failed"));
    if (loss_hist) loss_hist[e] = acc / ((double)steps_per_epoch * B);
  }
  s->step += total;
  return release(HJG_OK);
}

int hjg_surrogate_sweep(hjg_ctx* ctx, hjg_surrogate* s, const hjg_problem* p, int64_t Q, const float* x, double t,
                        int32_t N_s, int32_t K_s, int32_t N_fb, int32_t K_fb, double tol, uint32_t time_step,
                        float* v, float* grad, uint8_t* fell_back, int64_t* n_fallback, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_surrogate_sweep");
  if (!ctx || !s || !p || !n_fallback) return fail(HJG_EINVAL, "NULL argument");
  if (p->n != s->n) return fail(HJG_EINVAL, "problem dimension differs from the surrogate's");
  if (Q < 0) return fail(HJG_EINVAL, "Q must be >= 0");
  if (!(tol > 0)) return fail(HJG_EINVAL, "tol must be > 0 (it decides the fallback)");
  *n_fallback = 0;
  if (Q == 0) return HJG_OK;
  if (!x || !v || !grad || !fell_back) return fail(HJG_EINVAL, "x, v, grad and fell_back are required");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc;
  const int n = s->n;
  if ((rc = grow(s->sv, Q * 4)) || (rc = grow(s->sg, (size_t)Q * n * 4)) || (rc = grow(s->tq, Q * 4)) ||
      (rc = grow(s->index, Q * 4)) || (rc = grow(s->bcount, ((Q + 255) / 256 + 1) * 4)) || (rc = grow(s->total, 64)))
    return rc;
  // 1. the surrogate's value and gradient at (x, t)
  SG_HIP(launch_fill((float*)s->tq.p, (float)t, Q, st));
  if ((rc = hjg_surrogate_predict(s, Q, x, (const float*)s->tq.p, (float*)s->sv.p, (float*)s->sg.p, st))) return rc;
  // 2. Picard from the warm start (v^(0), p^(0)) = surrogate; the per-state
  //    relative change of the last iteration decides the fallback
  rc = hjg_picard_sweep(ctx, p, Q, x, t, N_s, K_s, tol, time_step, (const float*)s->sg.p, (const float*)s->sv.p, v,
                        grad, nullptr, nullptr, fell_back, nullptr, nullptr, hip_stream);
  // non-finite states (a non-finite surrogate output, say) carry the flag
  // and are solved again below; the final outputs are checked at the end
  if (rc < 0 && rc != HJG_ENONFINITE) return rc;
  // 3. plain Monte Carlo (no warm start) on the flagged states
  int nb = 0;
  SG_HIP(launch_compact_count(fell_back, Q, (int*)s->bcount.p, &nb, st));
  SG_HIP(launch_compact_scan((int*)s->bcount.p, nb, (int*)s->total.p, st));
  SG_HIP(launch_compact_write(fell_back, Q, (const int*)s->bcount.p, (int*)s->index.p, st));
  int count = 0;
  SG_HIP(hipMemcpyAsync(&count, s->total.p, 4, hipMemcpyDeviceToHost, st));
  SG_HIP(hipStreamSynchronize(st));
  *n_fallback = count;
  if (count > 0) {
    if ((rc = grow(s->xfb, (size_t)count * n * 4)) || (rc = grow(s->vfb, (size_t)count * 4)) ||
        (rc = grow(s->gfb, (size_t)count * n * 4)))
      return rc;
    SG_HIP(launch_gather_soa(x, n, Q, (const int*)s->index.p, count, (float*)s->xfb.p, st));
    rc = hjg_picard_sweep(ctx, p, count, (const float*)s->xfb.p, t, N_fb, K_fb, 0.0, time_step, nullptr, nullptr,
                          (float*)s->vfb.p, (float*)s->gfb.p, nullptr, nullptr, nullptr, nullptr, nullptr, hip_stream);
    if (rc < 0) return rc;
    SG_HIP(launch_scatter_soa((const float*)s->vfb.p, 1, count, (const int*)s->index.p, Q, v, st));
    SG_HIP(launch_scatter_soa((const float*)s->gfb.p, n, count, (const int*)s->index.p, Q, grad, st));
  }
  int* flag = (int*)s->total.p + 4;
  int host = 0;
  SG_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  SG_HIP(launch_finite_check(v, Q, flag, st));
  SG_HIP(launch_finite_check(grad, Q * n, flag, st));
  SG_HIP(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SG_HIP(hipStreamSynchronize(st));
  if (host) return fail(HJG_ENONFINITE, "non-finite value or gradient after the plain fallback");
  return HJG_OK;
}

// One time-marching step: Algorithm 1 over the horizon dt whose datum is the
// surrogate's value at the previous time (rows of a query chunk go through
// the network in one forward pass; the Picard bookkeeping is the sweep's).
int hjg_surrogate_tube_step(hjg_ctx* ctx, hjg_surrogate* s, const hjg_problem* p, int64_t Q, const float* x,
                            double t_prev, double dt, int32_t N, int32_t K, double tol, uint32_t time_step,
                            float* v, float* grad, float* c_out, float* ess, double* resid_hist,
                            int32_t* iters_done, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_surrogate_tube_step");
  if (!ctx || !s) return fail(HJG_EINVAL, "context or surrogate is NULL");
  int rc = detail::check_problem(p);
  if (rc) return rc;
  if (p->n != s->n) return fail(HJG_EINVAL, "problem dimension differs from the surrogate's");
  if (p->sample_mode != HJG_S_CRN_STEP)
    return fail(HJG_EUNSUPPORTED, "the time-marching step draws from a common table (sample_mode = crn_step)");
  if (Q < 0 || Q > ((int64_t)1 << 30)) return fail(HJG_EINVAL, "Q must be in [0, 2^30]");
  if (!(std::isfinite(t_prev) && t_prev >= 0)) return fail(HJG_EINVAL, "t_prev must be finite and >= 0");
  if (!(std::isfinite(dt) && dt > 0)) return fail(HJG_EINVAL, "dt must be finite and > 0");
  if (N < 1 || N > kTubeMaxSamples) return fail(HJG_EINVAL, "N must be in [1, 2^21]");
  if (K < 1 || K > 255) return fail(HJG_EINVAL, "K must be in [1, 255]");
  if (time_step >= 256) return fail(HJG_EINVAL, "time_step must be < 256");
  if (!(std::isfinite(tol) && tol >= 0)) return fail(HJG_EINVAL, "tol must be finite and >= 0");
  if (iters_done) *iters_done = 0;
  if (Q == 0) return HJG_OK;
  if (!x || !v || !grad) return fail(HJG_EINVAL, "x, v and grad are required");
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = s->n;
  const bool bf16 = p->sample_bf16 != 0;
  const int64_t tstride = (N + 63) / 64 * 64;
  const int64_t nblocks = (Q + kThreads - 1) / kThreads;
  int64_t rows_max = kTubeRowsPerChunk;
  if (const char* e = std::getenv("HJG_TUBE_ROWS")) rows_max = std::max<int64_t>(1, std::atoll(e));
  const int64_t Qc = std::max<int64_t>(1, std::min<int64_t>(Q, rows_max / N));
  // small networks run fused (HJG_TUBE_FUSED=0 forces the row-by-row form, for comparison)
  const char* fe = std::getenv("HJG_TUBE_FUSED");
  const bool fused = !(fe && fe[0] == '0') && s->width == kTubeFusedWidth && s->in_p == kTubeFusedInP &&
                     s->depth <= kTubeFusedMaxDepth && n <= kTubeFusedMaxN;
  if ((rc = grow(s->mt_table, (size_t)n * tstride * (bf16 ? 2 : 4))) || (rc = grow(s->mt_zbar, kMaxN * 8)) ||
      (rc = grow(s->mt_c, Q * 4)) || (rc = grow(s->mt_th, (size_t)Q * n * 4)) || (rc = grow(s->mt_vprev, Q * 4)) ||
      (rc = grow(s->mt_pm, Q * 4)) || (rc = grow(s->mt_pS, Q * 8)) || (rc = grow(s->mt_pS2, Q * 8)) ||
      (rc = grow(s->mt_pG, (size_t)Q * n * 4)) || (rc = grow(s->mt_block, nblocks * 24)) ||
      (rc = grow(s->mt_resid, (size_t)K * 8)) || (rc = grow(s->mt_ctrl, 64)) || (rc = grow(s->tq, Q * 4)) ||
      (!fused && (rc = ensure_batch(s, Qc * N, false))))
    return rc;
  // the common table of (problem, time step) and its column mean
  const uint32_t k0 = (uint32_t)(p->seed & 0xFFFFFFFFu), k1 = (uint32_t)(p->seed >> 32);
  SG_HIP(launch_table(n, tstride, tstride, k0, k1, detail::make_tag(p->problem_id, time_step, 0), bf16,
                      s->mt_table.p, st));
  if (p->grad_cv) SG_HIP(launch_zbar(n, N, tstride, bf16, s->mt_table.p, (double*)s->mt_zbar.p, st));
  // warm start: the surrogate's value and gradient at (x, t_prev)
  SG_HIP(launch_fill((float*)s->tq.p, (float)t_prev, Q, st));
  if ((rc = hjg_surrogate_predict(s, Q, x, (const float*)s->tq.p, (float*)s->mt_vprev.p, grad, st))) return rc;

  const float sigma = (float)std::sqrt(2.0 * p->nu * dt);
  int* done = (int*)s->mt_ctrl.p;
  int* iters = done + 1;
  int* nonfinite = done + 2;
  float* th = p->tilt ? (float*)s->mt_th.p : nullptr;
  hjg_problem pi = *p;              // the terminal datum is not used: a harmless one for init
  pi.datum = HJG_L_HALF_SQNORM;
  pi.datum_aux = nullptr;
  InitArgs in{};
  in.n = n;
  in.Q = Q;
  in.K = K;
  in.sigma = sigma;
  in.x = x;
  in.p0 = grad;
  in.v0 = (const float*)s->mt_vprev.p;
  in.dp = detail::datum_params(&pi);
  in.hp = detail::ham_params(p);
  in.tilt = p->tilt;
  in.vprev = (float*)s->mt_vprev.p;
  in.p = grad;
  in.c = (float*)s->mt_c.p;
  in.th = th;
  in.done = done;
  in.iters = iters;
  in.nonfinite = nonfinite;
  in.resid = (double*)s->mt_resid.p;
  SG_HIP(launch_init(in, st));
  const Partials part{(float*)s->mt_pm.p, (double*)s->mt_pS.p, (double*)s->mt_pS2.p, (float*)s->mt_pG.p, nullptr};
  TubeFusedArgs fa{};
  if (fused) {
    fa.n = n;
    fa.Q = Q;
    fa.N = N;
    fa.depth = s->depth;
    fa.x = x;
    fa.theta = th;
    fa.sigma = sigma;
    fa.table = s->mt_table.p;
    fa.tstride = tstride;
    fa.bf16 = bf16;
    fa.t_prev = (float)t_prev;
    fa.mean = nrm(s, 0);
    fa.stdv = nrm(s, 1);
    for (int l = 0; l <= s->depth; ++l) {
      fa.W[l] = (const __bf16*)s->Wb[l].p;
      fa.b[l] = (const float*)s->w.p + s->boff[l];
    }
    fa.omean = nrm(s, 2);
    fa.ostd = nrm(s, 3);
    fa.c = (const float*)s->mt_c.p;
    fa.part = part;
    fa.done = done;
  }
  for (int it = 0; it < K; ++it) {
    if (fused) SG_HIP(launch_tube_fused(fa, st));
    for (int64_t q0 = 0; q0 < Q && !fused; q0 += Qc) {
      const int64_t qc = std::min<int64_t>(Qc, Q - q0);
      TubePointsArgs a{};
      a.n = n;
      a.Q = Q;
      a.q0 = q0;
      a.Qc = qc;
      a.N = N;
      a.x = x;
      a.theta = th;
      a.sigma = sigma;
      a.table = s->mt_table.p;
      a.tstride = tstride;
      a.bf16 = bf16;
      a.t_prev = (float)t_prev;
      a.mean = nrm(s, 0);
      a.stdv = nrm(s, 1);
      a.ld = s->in_p;
      a.X0 = (__bf16*)s->X0.p;
      a.done = done;
      SG_HIP(launch_tube_points(a, st));
      if ((rc = forward(s, qc * N, false, st))) return rc;
      TubeLseArgs l{};
      l.n = n;
      l.Q = Q;
      l.q0 = q0;
      l.Qc = qc;
      l.N = N;
      l.c = (const float*)s->mt_c.p;
      l.theta = th;
      l.sigma = sigma;
      l.table = s->mt_table.p;
      l.tstride = tstride;
      l.bf16 = bf16;
      l.Y = (const float*)s->Y.p;
      l.ldy = s->out_p;
      l.omean = nrm(s, 2);
      l.ostd = nrm(s, 3);
      l.part = part;
      l.done = done;
      SG_HIP(launch_tube_lse(l, st));
    }
    FinalizeArgs f{};
    f.n = n;
    f.Q = Q;
    f.N = N;
    f.splits = 1;
    f.sigma = sigma;
    f.x = x;
    f.c = (const float*)s->mt_c.p;
    f.theta = th;
    f.part = part;
    f.cv = p->grad_cv;
    f.fresh = 0;
    f.zbar_tab = (const double*)s->mt_zbar.p;
    f.v = v;
    f.grad = grad;
    f.ess = ess;
    f.picard = 1;
    f.vprev = (float*)s->mt_vprev.p;
    f.c_out = c_out;
    f.flags = nullptr;
    f.tol = (float)tol;
    f.vfloor = (float)(1e-2 * std::sqrt(2.0 * p->nu * dt) * std::sqrt((double)n));
    f.blockpart = (double*)s->mt_block.p;
    f.c_next = (float*)s->mt_c.p;
    f.th_next = th;
    f.hp = in.hp;
    f.done = done;
    SG_HIP(launch_finalize(f, st));
    ReduceArgs r{};
    r.nblocks = (int)nblocks;
    r.blockpart = (const double*)s->mt_block.p;
    r.k = it;
    r.tol = (float)tol;
    r.resid = (double*)s->mt_resid.p;
    r.done = done;
    r.iters = iters;
    r.nonfinite = nonfinite;
    SG_HIP(launch_reduce(r, st));
    int flag = 0;
    SG_HIP(hipMemcpyAsync(&flag, done, 4, hipMemcpyDeviceToHost, st));
    SG_HIP(hipStreamSynchronize(st));
    if (flag) break;
  }
  int32_t ctl[3] = {0, 0, 0};
  SG_HIP(hipMemcpyAsync(ctl, done, sizeof(ctl), hipMemcpyDeviceToHost, st));
  if (resid_hist) SG_HIP(hipMemcpyAsync(resid_hist, s->mt_resid.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
  SG_HIP(hipStreamSynchronize(st));
  if (iters_done) *iters_done = ctl[1];
  if (ctl[2])
    return fail(HJG_ENONFINITE, std::to_string(ctl[2]) + " states have a non-finite value or gradient");
  return HJG_OK;
}

}  // extern "C"
