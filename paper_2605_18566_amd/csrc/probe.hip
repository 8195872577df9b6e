// Measurement helper: the issue rate of independent full-rate float32 FMAs
// at a given number of resident waves per SIMD.  The pair loop's roofline is
// priced against the chip's float32 vector peak (two wave-level FMA
// instructions per compute unit and clock); this probe measures how much of
// that rate plain FMAs reach at the occupancy a kernel runs at.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "hjg.h"
#include "internal.h"

namespace {

constexpr int kChains = 12;   // independent FMA chains per lane
constexpr int kUnroll = 8;    // chain steps per loop iteration

int fail(int code, const std::string& msg) { return hjg_internal_fail(code, msg.c_str()); }

// One block of 4 waves (one per SIMD); each lane runs kChains independent
// FMA chains.  Each wave records its elapsed shader-clock and 100 MHz
// real-time ticks around the loop.
// FORM 0: acc = acc * s + s (three-operand FMA with a scalar operand);
// FORM 1: acc = acc + a * b with a, b per lane (accumulating FMA);
// FORM 2: acc = acc * a (multiply);
// FORM 3: acc = acc * a + b with a, b per lane (three-operand FMA, vector operands);
// FORM 4: acc = acc + s * a (accumulating FMA with a scalar operand);
// FORM 5: acc = acc + s (add with a scalar operand);
// FORM 6: acc = min(acc, a, b) (three-input minimum);
// FORM 7: forms 0 and 1 on alternate chains (half the instructions read a
// scalar operand, as in the pair loop's offsets and squares).
// FORMS 8-10 fix the order and registers in inline assembly (vector-ALU
// instructions only), four instructions per step alternating a three-operand
// FMA with a scalar operand (S) and an accumulating FMA of vector registers
// (F), to separate the effect of dependences:
// FORM 8: S F S F, all independent;
// FORM 9: each F reads the result of the S just before it;
// FORM 10: each F reads the result of the S two before it, and the next S
// overwrites the register that F read (the pair loop's offset-square
// pattern).
// FORMS 11 and 12: forms 1 and 10 with the kernel's register allocation
// raised to 256 vector registers (at most two waves per SIMD), as in the
// pair loop.
template <int FORM>
__global__ __launch_bounds__(256) void valu_probe_kernel(int32_t iters, float mul, float add, float* sink,
                                                         unsigned long long* ticks) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = 1.0f + 1e-3f * (float)(lane + k);
  const float va = mul + 1e-9f * (float)lane, vb = add * (1.0f + 1e-9f * (float)lane);
  if constexpr (FORM >= 11) asm volatile("; holds the top register" ::: "v255");
  const unsigned long long c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if constexpr (FORM == 0) acc[k] = fmaf(acc[k], mul, add);
        else if constexpr (FORM == 1 || FORM == 11) acc[k] = fmaf(va, vb, acc[k]);
        else if constexpr (FORM == 2) acc[k] = acc[k] * va;
        else if constexpr (FORM == 3) acc[k] = fmaf(acc[k], va, vb);
        else if constexpr (FORM == 4) acc[k] = fmaf(mul, va, acc[k]);
        else if constexpr (FORM == 5) acc[k] = acc[k] + add;
        else if constexpr (FORM == 6) acc[k] = fminf(fminf(acc[k], va), vb);
        else if constexpr (FORM == 7) acc[k] = (k & 1) ? fmaf(va, vb, acc[k]) : fmaf(acc[k], mul, add);
        else if (k % 4 == 0) {
          if constexpr (FORM == 8)
            asm volatile("v_fma_f32 %0, %6, %4, %5\n\tv_fmac_f32 %1, %4, %5\n\t"
                         "v_fma_f32 %2, %6, %4, %5\n\tv_fmac_f32 %3, %4, %5"
                         : "+v"(acc[k]), "+v"(acc[k + 1]), "+v"(acc[k + 2]), "+v"(acc[k + 3])
                         : "v"(va), "v"(vb), "s"(mul));
          else if constexpr (FORM == 9)
            asm volatile("v_fma_f32 %0, %6, %4, %5\n\tv_fmac_f32 %1, %0, %0\n\t"
                         "v_fma_f32 %2, %6, %4, %5\n\tv_fmac_f32 %3, %2, %2"
                         : "+v"(acc[k]), "+v"(acc[k + 1]), "+v"(acc[k + 2]), "+v"(acc[k + 3])
                         : "v"(va), "v"(vb), "s"(mul));
          else if constexpr (FORM == 10 || FORM == 12)
            asm volatile("v_fma_f32 %0, %6, %4, %5\n\tv_fmac_f32 %1, %2, %2\n\t"
                         "v_fma_f32 %2, %6, %4, %5\n\tv_fmac_f32 %3, %0, %0"
                         : "+v"(acc[k]), "+v"(acc[k + 1]), "+v"(acc[k + 2]), "+v"(acc[k + 3])
                         : "v"(va), "v"(vb), "s"(mul));
        }
      }
  }
  const unsigned long long c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += acc[k];
  sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
  if (lane == 0) {
    ticks[((int64_t)blockIdx.x * 4 + wave) * 2] = c1 - c0;
    ticks[((int64_t)blockIdx.x * 4 + wave) * 2 + 1] = r1 - r0;
  }
}

}  // namespace

int hjg_probe_valu_rate(int32_t waves_per_simd, int32_t iters, int32_t form, double* instr_per_cu_clock,
                        double* clock_ghz, void* hip_stream) {
  const hjg::detail::TraceRange trace_("hjg_probe_valu_rate");
  if (!instr_per_cu_clock || !clock_ghz) return fail(HJG_EINVAL, "NULL argument");
  if (waves_per_simd < 1 || waves_per_simd > 8) return fail(HJG_EINVAL, "waves_per_simd must be in [1, 8]");
  if (iters < 1 || iters > (1 << 24)) return fail(HJG_EINVAL, "iters must be in [1, 2^24]");
  if (form < 0 || form > 12) return fail(HJG_EINVAL, "form must be in [0, 12]");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || ncu < 1)
    return fail(HJG_EHIP, "cannot query the compute-unit count");
  const int blocks = ncu * waves_per_simd;   // blocks of 4 waves: waves_per_simd blocks per compute unit
  float* sink = nullptr;
  unsigned long long* ticks = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&](int code) {
    if (sink) (void)hipFree(sink);
    if (ticks) (void)hipFree(ticks);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return code;
  };
  if (hipMalloc(&sink, (size_t)blocks * 256 * sizeof(float)) != hipSuccess ||
      hipMalloc(&ticks, (size_t)blocks * 8 * sizeof(unsigned long long)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return cleanup(fail(HJG_ENOMEM, "probe workspace allocation failed"));
  // one warm-up launch, then the timed one
  auto launch = [&](int it) {
    switch (form) {
      case 0: valu_probe_kernel<0><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 1: valu_probe_kernel<1><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 2: valu_probe_kernel<2><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 3: valu_probe_kernel<3><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 4: valu_probe_kernel<4><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 5: valu_probe_kernel<5><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 6: valu_probe_kernel<6><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 7: valu_probe_kernel<7><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 8: valu_probe_kernel<8><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 9: valu_probe_kernel<9><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 10: valu_probe_kernel<10><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      case 11: valu_probe_kernel<11><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
      default: valu_probe_kernel<12><<<blocks, 256, 0, st>>>(it, 0.9999f, 1e-4f, sink, ticks); break;
    }
  };
  launch(std::max(1, iters / 16));
  (void)hipEventRecord(e0, st);
  launch(iters);
  (void)hipEventRecord(e1, st);
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return cleanup(fail(HJG_EHIP, "valu_probe_kernel failed"));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  std::vector<unsigned long long> h((size_t)blocks * 8);
  if (hipMemcpy(h.data(), ticks, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(HJG_EHIP, "probe read-back failed"));
  // shader clock from the waves' own counters: clock ticks per 100 MHz tick
  double cyc = 0.0, rt = 0.0;
  for (int w = 0; w < blocks * 4; ++w) {
    cyc += (double)h[2 * w];
    rt += (double)h[2 * w + 1];
  }
  if (!(rt > 0.0) || !(ms > 0.f)) return cleanup(fail(HJG_EHIP, "probe timing failed"));
  const double hz = cyc / rt * 1e8;
  const double instr = (double)blocks * 4.0 * (double)iters * kUnroll * kChains;
  *clock_ghz = hz * 1e-9;
  *instr_per_cu_clock = instr / ((double)ms * 1e-3 * hz * (double)ncu);
  return cleanup(HJG_OK);
}
