// Small device utilities: a fill kernel used instead of hipMemsetAsync so
// that the library's calls stay safe under stream capture.
#include "vg_internal.h"

namespace vg {
namespace {

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    p[q] = v;
}

}  // namespace

hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace vg
