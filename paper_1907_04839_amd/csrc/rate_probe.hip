// Issue-rate probes for gfx950: the measured ceilings beside the published
// peak.  MI355X's published FP32 vector peak counts packed FP32 FMAs, which
// this build never emits; these kernels measure what plain (non-packed)
// instructions of the kinds the pair loops use reach on the chip:
//
//   kind 0  FP32 FMA (v_fma_f32) with every operand in VGPRs
//   kind 1  FP32 FMA with one SGPR operand (the pair loops read the j
//           landmark from SGPRs)
//   kind 2  v_exp_f32 (2^x, the Gaussian of every pair)
//   kind 3  v_fma_f64
//   kind 4  v_mul_f32 with VGPR operands
//   kind 5  v_mfma_f32_16x16x4_f32 (4 independent accumulators per wave);
//           the rate counts one lane-operation per lane per MFMA (an MFMA is
//           16 x 16 x 4 = 1024 FMAs, i.e. 16 per lane)
//   kind 6  the same 4 MFMAs per round interleaved with 28 independent FP32
//           FMAs with VGPR operands; the rate counts one per lane per round,
//           to compare with kinds 0 and 5 run alone
//
// Each lane runs 8 independent dependency chains (enough to cover the ALU
// latency) for `iters` rounds; a launch has 8 waves per SIMD of the chip.
// The benchmark loads this library on its own; the shooting library does not
// use it.
#include <hip/hip_runtime.h>

namespace {

constexpr int kChains = 8;
constexpr int kBlock = 256;

// b, c: per-lane values (VGPRs) for kind 0 and 4; kernel arguments (SGPRs)
// for kind 1.
__global__ __launch_bounds__(kBlock) void k_fma_v(const float* __restrict__ bc, int iters,
                                                  float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const float b = bc[2 * t], c = bc[2 * t + 1];
  float a[kChains];
  for (int k = 0; k < kChains; ++k) a[k] = 0.25f * (float)(k + 1) + 1e-3f * (float)threadIdx.x;
#pragma unroll 4
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = s;
}

__global__ __launch_bounds__(kBlock) void k_fma_s(float b, float c, int iters,
                                                  float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  float a[kChains];
  for (int k = 0; k < kChains; ++k) a[k] = 0.25f * (float)(k + 1) + 1e-3f * (float)threadIdx.x;
#pragma unroll 4
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = s;
}

// a <- 2^(-a): a bounded chain (fixed point near 0.64), one v_exp_f32 with a
// negate modifier per step, as in the pair loops.
__global__ __launch_bounds__(kBlock) void k_exp(int iters, float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  float a[kChains];
  for (int k = 0; k < kChains; ++k) a[k] = 0.1f * (float)(k + 1) + 1e-4f * (float)threadIdx.x;
#pragma unroll 4
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = s;
}

__global__ __launch_bounds__(kBlock) void k_fma64(const float* __restrict__ bc, int iters,
                                                  float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const double b = bc[2 * t], c = bc[2 * t + 1];
  double a[kChains];
  for (int k = 0; k < kChains; ++k) a[k] = 0.25 * (k + 1) + 1e-3 * threadIdx.x;
#pragma unroll 4
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
  double s = 0.0;
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = (float)s;
}

__global__ __launch_bounds__(kBlock) void k_mul_v(const float* __restrict__ bc, int iters,
                                                  float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const float b = bc[2 * t];
  float a[kChains];
  for (int k = 0; k < kChains; ++k) a[k] = 0.25f * (float)(k + 1) + 1e-3f * (float)threadIdx.x;
#pragma unroll 4
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = a[k] * b;
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = s;
}

using F4 = float __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_mfma(const float* __restrict__ bc, int iters,
                                                 float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const float a = bc[2 * t] + 1.0f, b = bc[2 * t + 1] + 0.5f;
  F4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
#pragma unroll 2
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
  }
  const F4 c = c0 + c1 + c2 + c3;
  out[t] = c[0] + c[1] + c[2] + c[3];
}

__global__ __launch_bounds__(kBlock) void k_mfma_valu(const float* __restrict__ bc, int iters,
                                                      float* __restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const float a = bc[2 * t] + 1.0f, b = bc[2 * t + 1] + 0.5f;
  F4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  float v[7];
  for (int k = 0; k < 7; ++k) v[k] = 0.25f * (float)(k + 1) + 1e-3f * (float)threadIdx.x;
#pragma unroll 2
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = fmaf(v[k], b, a);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = fmaf(v[k], b, a);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = fmaf(v[k], b, a);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = fmaf(v[k], b, a);
  }
  const F4 c = c0 + c1 + c2 + c3;
  float s = c[0] + c[1] + c[2] + c[3];
  for (int k = 0; k < 7; ++k) s += v[k];
  out[t] = s;
}

}  // namespace

extern "C" {

// Runs probe `kind` (0-6) with `iters` rounds of 8 chains per lane on a grid
// of `blocks` workgroups of 256 threads, `reps` timed launches after one
// warm-up; writes the lane-operations per second (one FMA, multiply or exp
// per lane per chain step) to *rate.  Returns a hipError_t (0 = success).
int rate_probe_run(int kind, int blocks, int iters, int reps, double* rate) {
  if (kind < 0 || kind > 6 || blocks < 1 || iters < 1 || reps < 1 || !rate) return 1;
  const size_t threads = (size_t)blocks * kBlock;
  float *bc = nullptr, *out = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipMalloc(&bc, 2 * threads * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&out, threads * sizeof(float));
  if (e == hipSuccess) e = hipMemset(bc, 0, 2 * threads * sizeof(float));
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  auto launch = [&]() {
    switch (kind) {
      case 0: k_fma_v<<<blocks, kBlock>>>(bc, iters, out); break;
      case 1: k_fma_s<<<blocks, kBlock>>>(0.999f, 1e-3f, iters, out); break;
      case 2: k_exp<<<blocks, kBlock>>>(iters, out); break;
      case 3: k_fma64<<<blocks, kBlock>>>(bc, iters, out); break;
      case 4: k_mul_v<<<blocks, kBlock>>>(bc, iters, out); break;
      case 5: k_mfma<<<blocks, kBlock>>>(bc, iters, out); break;
      default: k_mfma_valu<<<blocks, kBlock>>>(bc, iters, out); break;
    }
  };
  if (e == hipSuccess) {
    launch();
    e = hipEventRecord(ev[0], nullptr);
  }
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  const int per_round = kind == 5 ? 4 : kind == 6 ? 1 : kChains;
  if (e == hipSuccess)
    *rate = (double)threads * iters * per_round * reps / (ms * 1e-3);
  for (hipEvent_t v : ev)
    if (v) (void)hipEventDestroy(v);
  if (bc) (void)hipFree(bc);
  if (out) (void)hipFree(out);
  return (int)e;
}

}  // extern "C"
