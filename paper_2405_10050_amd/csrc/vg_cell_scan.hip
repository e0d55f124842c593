// Launchers of the Monte-Carlo cell scan (kernels in vg_cell_scan.h): the
// directions-as-input instances and the persistent batched scan.  The
// instances that draw the directions on the device are compiled separately
// (vg_cell_scan_gen.hip).
#include "vg_cell_scan.h"

namespace vg {
namespace {
// ------------------------------------------------------- persistent batches
// Uneven batches of clouds: workgroups take (cloud, cell, ray chunk) items
// from a device counter, in the order of the item table (largest clouds
// first), until the counter passes the end of the launch's item range.  One
// launch serves one register class of K extents (FP32: K pairs {1,2}, {3,4},
// {5,6}, {7,8}; BF16x3: each K group alone): a kernel that inlined every
// extent would be allocated the registers of the largest and lose occupancy
// on the small ones.
template <int K, int KHI, int C, int WAVES>
__device__ __forceinline__ void dispatch_fp32(int kp, const CellScanArgs &a, int64_t cell, int chunk,
                                              float *l, float *red) {
  if constexpr (K < KHI) {
    if (kp == K) {
      scan_fp32_item<K, C, WAVES, false>(a, cell, chunk, l, red);
      return;
    }
    dispatch_fp32<K + 1, KHI, C, WAVES>(kp, a, cell, chunk, l, red);
  } else {
    scan_fp32_item<K, C, WAVES, false>(a, cell, chunk, l, red);
  }
}

template <int C, int WAVES, bool BF16, int KLO, int KHI>
__global__ __launch_bounds__(WAVES * 64) void cell_scan_batched_kernel(const BatchProblem *__restrict__ probs,
                                                                      int np, int64_t first,
                                                                      int64_t last,
                                                                      unsigned long long *next) {
  constexpr int NT = WAVES * 64;
  constexpr size_t FP32_LDS = Fp32Tile<KHI, WAVES>::FLOATS * sizeof(float);
  constexpr size_t BF16_LDS = NT * (Bf16Pack<KHI>::KT / 8) * sizeof(bf16x8);
  __shared__ __align__(16) unsigned char raw[BF16 ? BF16_LDS : FP32_LDS];
  __shared__ float red[NT];
  __shared__ long long item_s;
  for (;;) {
    __syncthreads();  // the previous item is finished
    if (threadIdx.x == 0) item_s = first + (long long)atomicAdd(next, 1ull);
    __syncthreads();
    const long long item = item_s;
    if (item >= last) break;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].item_begin <= item)
        lo = mid;
      else
        hi = mid - 1;
    }
    const CellScanArgs a = probs[lo].a;
    const int64_t local = item - probs[lo].item_begin;
    const int64_t cell = local / a.wg_per_cell;
    const int chunk = (int)(local - cell * a.wg_per_cell);
    if constexpr (BF16) {
      scan_bf16x3_item<KHI, C, WAVES, false>(a, cell, chunk, reinterpret_cast<bf16x8 *>(raw), red);
    } else {
      dispatch_fp32<KLO, KHI, C, WAVES>((a.d + 1) >> 1, a, cell, chunk, reinterpret_cast<float *>(raw),
                                        red);
    }
  }
}

template <int C, int WAVES>
hipError_t launch_kq(const CellScanArgs &a, hipStream_t s, int grid) {
  return a.dirs ? launch_kq_g<C, WAVES, false>(a, s, grid) : launch_cells_gen(a, true, C * WAVES * 32, grid, s);
}

template <int C, int WAVES>
hipError_t launch_kp(const CellScanArgs &a, hipStream_t s, int grid) {
  return a.dirs ? launch_kp_g<C, WAVES, false>(a, s, grid) : launch_cells_gen(a, false, C * WAVES * 32, grid, s);
}

}  // namespace

int cell_scan_rays_per_wg(int R) {
  if (R >= 1024) return 1024;
  if (R >= 512) return 512;
  if (R >= 256) return 256;
  if (R >= 128) return 128;
  return 64;
}

hipError_t launch_cell_scan_fp32(const CellScanArgs &a0, hipStream_t s) {
  CellScanArgs a = a0;
  const int rw = cell_scan_rays_per_wg(a.R);
  a.wg_per_cell = (a.R + rw - 1) / rw;
  const int64_t grid64 = a.n * a.wg_per_cell;
  if (grid64 <= 0) return hipSuccess;
  if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
  const int grid = (int)grid64;
  switch (rw) {
    case 1024: return launch_kp<4, 8>(a, s, grid);
    case 512: return launch_kp<2, 8>(a, s, grid);
    case 256: return launch_kp<2, 4>(a, s, grid);
    case 128: return launch_kp<1, 4>(a, s, grid);
    default: return launch_kp<1, 2>(a, s, grid);
  }
}

hipError_t launch_cell_scan_bf16x3(const CellScanArgs &a0, hipStream_t s) {
  CellScanArgs a = a0;
  const int rw = cell_scan_rays_per_wg(a.R);
  a.wg_per_cell = (a.R + rw - 1) / rw;
  const int64_t grid64 = a.n * a.wg_per_cell;
  if (grid64 <= 0) return hipSuccess;
  if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
  const int grid = (int)grid64;
  switch (rw) {
    case 1024: return launch_kq<4, 8>(a, s, grid);
    case 512: return launch_kq<2, 8>(a, s, grid);
    case 256: return launch_kq<2, 4>(a, s, grid);
    case 128: return launch_kq<1, 4>(a, s, grid);
    default: return launch_kq<1, 2>(a, s, grid);
  }
}

// Shapes of the persistent batched scan (rays per item = 32 * C * WAVES).
const BatchShape kBatchShapes[kNumBatchShapes] = {{1, 8}, {2, 4}, {4, 8}};

int batched_class(int d, bool bf16) {
  if (bf16) return d <= 5 ? 0 : (d <= 10 ? 1 : 2);
  return (((d + 1) >> 1) - 1) >> 1;  // K pairs {1,2} -> 0, {3,4} -> 1, {5,6} -> 2, {7,8} -> 3
}

namespace {

template <int C, int WAVES, bool BF16>
hipError_t launch_class(const BatchProblem *probs, int np, int64_t first, int64_t last,
                        unsigned long long *next, int cls, int grid, hipStream_t s) {
  dim3 g(grid), b(WAVES * 64);
  if constexpr (BF16) {
    switch (cls) {
      case 0: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, true, 1, 1>), g, b, 0, s, probs, np, first, last, next); break;
      case 1: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, true, 2, 2>), g, b, 0, s, probs, np, first, last, next); break;
      default: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, true, 3, 3>), g, b, 0, s, probs, np, first, last, next); break;
    }
  } else {
    switch (cls) {
      case 0: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, false, 1, 2>), g, b, 0, s, probs, np, first, last, next); break;
      case 1: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, false, 3, 4>), g, b, 0, s, probs, np, first, last, next); break;
      case 2: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, false, 5, 6>), g, b, 0, s, probs, np, first, last, next); break;
      default: hipLaunchKernelGGL((cell_scan_batched_kernel<C, WAVES, false, 7, 8>), g, b, 0, s, probs, np, first, last, next); break;
    }
  }
  return hipGetLastError();
}

template <int C, int WAVES, bool BF16>
int class_blocks_per_cu(int cls) {
  int nb = 0;
  hipError_t e;
  constexpr int NT = WAVES * 64;
  if constexpr (BF16) {
    switch (cls) {
      case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, true, 1, 1>, NT, 0); break;
      case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, true, 2, 2>, NT, 0); break;
      default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, true, 3, 3>, NT, 0); break;
    }
  } else {
    switch (cls) {
      case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, false, 1, 2>, NT, 0); break;
      case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, false, 3, 4>, NT, 0); break;
      case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, false, 5, 6>, NT, 0); break;
      default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cell_scan_batched_kernel<C, WAVES, false, 7, 8>, NT, 0); break;
    }
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace

hipError_t launch_cell_scan_batched(const BatchProblem *probs_dev, int np, int64_t first, int64_t last,
                                    unsigned long long *next, int shape, bool bf16, int cls, int grid,
                                    hipStream_t s) {
  if (last <= first) return hipSuccess;
  switch (shape) {
    case 0: return bf16 ? launch_class<1, 8, true>(probs_dev, np, first, last, next, cls, grid, s)
                        : launch_class<1, 8, false>(probs_dev, np, first, last, next, cls, grid, s);
    case 1: return bf16 ? launch_class<2, 4, true>(probs_dev, np, first, last, next, cls, grid, s)
                        : launch_class<2, 4, false>(probs_dev, np, first, last, next, cls, grid, s);
    default: return bf16 ? launch_class<4, 8, true>(probs_dev, np, first, last, next, cls, grid, s)
                         : launch_class<4, 8, false>(probs_dev, np, first, last, next, cls, grid, s);
  }
}

int batched_blocks_per_cu(int shape, bool bf16, int cls) {
  switch (shape) {
    case 0: return bf16 ? class_blocks_per_cu<1, 8, true>(cls) : class_blocks_per_cu<1, 8, false>(cls);
    case 1: return bf16 ? class_blocks_per_cu<2, 4, true>(cls) : class_blocks_per_cu<2, 4, false>(cls);
    default: return bf16 ? class_blocks_per_cu<4, 8, true>(cls) : class_blocks_per_cu<4, 8, false>(cls);
  }
}

}  // namespace vg
