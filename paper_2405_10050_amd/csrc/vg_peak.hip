// Measured peak rates of the three arithmetic pipes the library runs on:
// FP32 MFMA (v_mfma_f32_32x32x2f32, the FP32 cell scan), BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, the split-BF16x3 scan) and FP64 vector FMA (the
// recheck).  Each kernel keeps several independent accumulation chains per
// wave so that issue, not latency, bounds it, on a grid that fills every
// SIMD; the rate is the work of one launch over its HIP-event duration.
#include <algorithm>
#include <cstdio>

#include "vg_internal.h"

namespace vg {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kChains = 4;   // independent MFMA accumulators per wave
constexpr int kFmaChains = 8;  // independent FP64 FMA chains per lane

__global__ __launch_bounds__(256) void peak_fp32_mfma(int iters, float seed, float *out) {
  const float a = seed + (float)(threadIdx.x & 7), b = seed * 0.5f;
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[c][i] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[c][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void peak_bf16_mfma(int iters, float seed, float *out) {
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(seed + (float)e);
    b[e] = (__bf16)(seed * 0.25f);
  }
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[c][i] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[c][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void peak_fp64_fma(int iters, float seed, float *out) {
  double x[kFmaChains];
  const double m = 0.999999 + 1e-9 * (double)(threadIdx.x & 3), c0 = 1e-7 * (double)seed;
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) x[c] = (double)seed + c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) x[c] = __builtin_fma(x[c], m, c0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" int vg_peak_rate(vg_ctx *ctx, int kind, double *flops_per_s) {
  if (!ctx || !flops_per_s) return VG_EINVAL;
  ctx->err.clear();
  if (kind < 0 || kind > 2) {
    ctx->err = "kind outside {0, 1, 2}";
    return VG_EINVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return VG_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return VG_EDEVICE;
  // 8 waves per CU-SIMD pair: 2 workgroups of 4 waves per SIMD
  const int blocks = prop.multiProcessorCount * 8;
  const int threads = 256;
  float *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VG_OK;
  if (hipMalloc(&out, (size_t)blocks * threads * sizeof(float)) != hipSuccess) return VG_ENOMEM;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = VG_EDEVICE;
  // work per wave-iteration: chains x MFMA flops, or chains x 64 lanes x 2
  const double per_iter = kind == 0 ? kChains * 32.0 * 32 * 2 * 2
                        : kind == 1 ? kChains * 32.0 * 32 * 16 * 2
                                    : kFmaChains * 64.0 * 2;
  // about 50 ms per launch at the datasheet rates
  const int iters = kind == 0 ? 51200 : kind == 1 ? 102400 : 409600;
  double best = 0.0;
  for (int rep = 0; rep < 3 && rc == VG_OK; ++rep) {
    (void)hipEventRecord(e0, ctx->stream);
    if (kind == 0)
      hipLaunchKernelGGL(peak_fp32_mfma, dim3(blocks), dim3(threads), 0, ctx->stream, iters, 1.0f, out);
    else if (kind == 1)
      hipLaunchKernelGGL(peak_bf16_mfma, dim3(blocks), dim3(threads), 0, ctx->stream, iters, 1.0f, out);
    else
      hipLaunchKernelGGL(peak_fp64_fma, dim3(blocks), dim3(threads), 0, ctx->stream, iters, 1.0f, out);
    if (hipGetLastError() != hipSuccess) rc = VG_EDEVICE;
    (void)hipEventRecord(e1, ctx->stream);
    float ms = 0.f;
    if (rc == VG_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = VG_EDEVICE;
    const double waves = (double)blocks * threads / 64.0;
    if (rc == VG_OK && ms > 0.f) best = std::max(best, waves * iters * per_iter / (ms * 1e-3));
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (rc == VG_OK) *flops_per_s = best;
  return rc;
}
