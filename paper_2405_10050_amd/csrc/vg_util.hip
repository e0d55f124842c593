// Small device utilities: a fill kernel used instead of hipMemsetAsync so
// that the library's calls stay safe under stream capture, and the checks of
// non-finite inputs (a count of bad node coordinates; the rays they or their
// own non-finite origin or direction invalidate answered NaN / -1).
#include "vg_internal.h"

namespace vg {
namespace {

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    p[q] = v;
}

__device__ __forceinline__ bool finite_f(float x) { return (__float_as_uint(x) & 0x7f800000u) != 0x7f800000u; }

__global__ __launch_bounds__(256) void check_finite_kernel(const float *__restrict__ x, int64_t count,
                                                          uint32_t *bad) {
  uint32_t local = 0;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < count; q += (int64_t)gridDim.x * 256)
    local += finite_f(x[q]) ? 0u : 1u;
  if (local) atomicAdd(bad, local);
}

__global__ __launch_bounds__(256) void finalize_bad_kernel(FinalizeArgs f) {
  const bool all = f.flags[CNT_BAD_NODES] != 0;
  if (!all && !f.u32 && !f.o32 && !f.u64 && !f.o64) return;
  uint32_t local = 0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < f.m; r += (int64_t)gridDim.x * 256) {
    bool bad = all;
    for (int k = 0; k < f.d && !bad; ++k) {
      if (f.u32 && !finite_f(f.u32[r * f.d + k])) bad = true;
      if (f.o32 && !finite_f(f.o32[r * f.d + k])) bad = true;
      if (f.u64 && !__builtin_isfinite(f.u64[r * f.d + k])) bad = true;
      if (f.o64 && !__builtin_isfinite(f.o64[r * f.d + k])) bad = true;
    }
    if (bad) {
      f.t_out[r] = __builtin_nanf("");
      f.idx_out[r] = -1;
      f.st_out[r] = VG_ST_BAD_INPUT;
      ++local;
    }
  }
  if (local) atomicAdd(f.bad_rays, local);
}

}  // namespace

hipError_t launch_check_finite(const float *x, int64_t count, uint32_t *bad, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, count, bad);
  return hipGetLastError();
}

hipError_t launch_finalize_bad(const FinalizeArgs &f, hipStream_t s) {
  if (f.m <= 0) return hipSuccess;
  int64_t blocks = (f.m + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(finalize_bad_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace vg
