// Scan order of the nodes for the Monte-Carlo cell scan.
//
// The cell scan visits every node for every ray of a cell (Algorithm 3 over
// eq. (t)), but a 32-node block whose bound on u.r~ is below every lane's
// current second-best value cannot change any ray's top two and is skipped
// (the skip is exact: the result is the one of the full scan).  Such blocks
// are frequent only when the nodes of a block lie close to each other in
// every coordinate, so the scan runs over a copy of the nodes sorted along a
// Morton (Z-order) curve of all their coordinates (up to 32), each scaled to
// the cloud's bounding box, and each cell starts at its own place in that
// order and works outwards: the blocks near x_i, which hold the rays'
// winners, come first and raise the second-best values before the far blocks
// are reached.  (A curve over only a few coordinates leaves each block spread
// over the full range of the others, and its bound loose.)
//
// The pass also records the bounding box and a bounding ball of every 128
// consecutive nodes of the sorted copy, from which the scan bounds whole
// chunks of nodes before loading them.
//
// The order is a pure function of the coordinates: the sort key is
// (Morton code << 32) | node index, unique per node, so any correct sort gives
// the same permutation.  Sort: bitonic over the next power of two of n (pads
// are all-ones keys), in LDS for spans up to 1024 and in global memory above;
// plain kernels only (no memset), so a caller may capture the pass in a
// hipGraph.
#include "vg_internal.h"

namespace vg {
namespace {

constexpr int kSortSpan = 1024;  // keys sorted in LDS by one workgroup
constexpr int kSortThreads = kSortSpan / 2;

// Order-preserving map of a float onto uint32 (for atomic min / max).
__device__ __forceinline__ uint32_t float_key(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// box[k] / box[d + k]: float_key of the minimum / maximum of coordinate k.
__global__ void cloud_box_init_kernel(int d, uint32_t *__restrict__ box) {
  for (int k = threadIdx.x; k < 2 * d; k += blockDim.x) box[k] = k < d ? 0xffffffffu : 0u;
}

// Bounding box of the cloud: per coordinate, a grid-stride min / max over the
// nodes (NaN ignored), reduced over the wave, then over the block's four
// waves in LDS, and one atomic per block (a few dozen blocks: the atomics on
// the 2d words would otherwise queue behind each other).
constexpr int kBoxBlocks = 64;
__global__ __launch_bounds__(256) void cloud_box_kernel(const float *__restrict__ nodes, int64_t n, int d,
                                                        uint32_t *__restrict__ box) {
  __shared__ float red[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < d; ++k) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const float v = nodes[i * d + k];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      red[0][wave] = lo;
      red[1][wave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      lo = fminf(fminf(red[0][0], red[0][1]), fminf(red[0][2], red[0][3]));
      hi = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
      atomicMin(box + k, float_key(lo));
      atomicMax(box + d + k, float_key(hi));
    }
    __syncthreads();
  }
}

// Morton code of the first m = min(d, 32) coordinates, 32 / m bits each,
// coordinate k scaled from [lo_k, hi_k] of the cloud's box (values outside,
// NaN and a degenerate or infinite extent map into the range).
__device__ __forceinline__ uint32_t morton_key(const float *x, int d, const uint32_t *box) {
  const int m = d < 32 ? d : 32;
  const int bits = 32 / m;
  const float cells = (float)(1u << bits);
  uint32_t code = 0;
  for (int b = bits - 1; b >= 0; --b) {
    for (int k = 0; k < m; ++k) {
      const float lo = key_float(box[k]), hi = key_float(box[d + k]);
      const float scale = hi > lo ? cells / (hi - lo) : 0.f;
      const float v = (x[k] - lo) * scale;
      const uint32_t q = v >= 1.f ? (v < cells ? (uint32_t)v : (1u << bits) - 1u) : 0u;
      code = (code << 1) | ((q >> b) & 1u);
    }
  }
  return code;
}

__global__ void order_keys_kernel(const float *__restrict__ nodes, int64_t n, int d, int64_t p2,
                                  const uint32_t *__restrict__ box, uint64_t *__restrict__ keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p2; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = i < n ? ((uint64_t)morton_key(nodes + i * d, d, box) << 32) | (uint64_t)i : ~0ull;
}

__device__ __forceinline__ void cmp_swap(uint64_t &a, uint64_t &b, bool asc) {
  if ((a > b) == asc) {
    const uint64_t t = a;
    a = b;
    b = t;
  }
}

// Bitonic stages (k, j) with j < kSortSpan over one span of kSortSpan keys in
// LDS.  k_first == 0: every stage k = 2 .. kSortSpan (the span is sorted in
// the direction its global position asks for); else the stages j = kSortSpan/2
// .. 1 of merge size k_first.
__global__ __launch_bounds__(kSortThreads) void bitonic_local_kernel(uint64_t *__restrict__ keys,
                                                                     int64_t k_first) {
  __shared__ uint64_t s[kSortSpan];
  const int64_t base = (int64_t)blockIdx.x * kSortSpan;
  const int t = threadIdx.x;
  s[t] = keys[base + t];
  s[t + kSortThreads] = keys[base + t + kSortThreads];
  __syncthreads();
  const int64_t k_lo = k_first ? k_first : 2;
  const int64_t k_hi = k_first ? k_first : kSortSpan;
  for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
    for (int j = (int)(k_first ? kSortSpan / 2 : k / 2); j > 0; j >>= 1) {
      const int i = 2 * t - (t & (j - 1));  // bit j of i is clear
      const bool asc = ((base + i) & k) == 0;
      uint64_t a = s[i], b = s[i + j];
      cmp_swap(a, b, asc);
      s[i] = a;
      s[i + j] = b;
      __syncthreads();
    }
  }
  keys[base + t] = s[t];
  keys[base + t + kSortThreads] = s[t + kSortThreads];
}

// One bitonic stage (k, j), j >= kSortSpan, in global memory.
__global__ void bitonic_global_kernel(uint64_t *__restrict__ keys, int64_t p2, int64_t k, int64_t j) {
  const int64_t half = p2 / 2;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < half; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = 2 * t - (t & (j - 1));
    const bool asc = (i & k) == 0;
    uint64_t a = keys[i], b = keys[i + j];
    cmp_swap(a, b, asc);
    keys[i] = a;
    keys[i + j] = b;
  }
}

__global__ void order_apply_kernel(const uint64_t *__restrict__ keys, const float *__restrict__ nodes, int64_t n,
                                   int d, int32_t *__restrict__ perm, int32_t *__restrict__ rank,
                                   float *__restrict__ xs) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = (int32_t)(keys[p] & 0xffffffffull);
    perm[p] = i;
    rank[i] = (int32_t)p;
    for (int k = 0; k < d; ++k) xs[p * d + k] = nodes[(int64_t)i * d + k];
  }
}

// Bounding box and bounding ball of each kOrderGroup consecutive nodes of
// xs: one wave per group, two nodes per lane, reductions over the lanes per
// coordinate.  The ball's centre is the group's mean (lane k keeps
// coordinate k, d <= 64) and its radius the largest distance of a node from
// it, rounded up by 2^-16 relative, far above the FP32 rounding of the
// squared distances (d + 2 roundings of 2^-24 each), so every node of the
// group lies in the stored ball.
__global__ __launch_bounds__(256) void order_boxes_kernel(const float *__restrict__ xs, int64_t n, int d,
                                                          float *__restrict__ aabb, float *__restrict__ ball) {
  const int lane = threadIdx.x & 63;
  const int64_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= order_groups(n)) return;
  const int64_t p0 = g * kOrderGroup;
  const int cnt = (int)(n - p0 < kOrderGroup ? n - p0 : kOrderGroup);
  float ck = 0.f;
  for (int k = 0; k < d; ++k) {
    float lo = __builtin_inff(), hi = -__builtin_inff(), sum = 0.f;
    for (int e = lane; e < cnt; e += 64) {
      const float v = xs[(p0 + e) * d + k];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
      sum += v;
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
      sum += __shfl_xor(sum, off);
    }
    if (lane == 0) {
      aabb[g * 2 * d + k] = lo;
      aabb[g * 2 * d + d + k] = hi;
    }
    if (lane == k) ck = sum / (float)cnt;
  }
  float r2 = 0.f;
  for (int e = lane; e < cnt; e += 64) {
    float s2 = 0.f;
    for (int k = 0; k < d; ++k) {
      const float diff = xs[(p0 + e) * d + k] - __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ck), k));
      s2 = __builtin_fmaf(diff, diff, s2);
    }
    r2 = fmaxf(r2, s2);
  }
  for (int off = 32; off > 0; off >>= 1) r2 = fmaxf(r2, __shfl_xor(r2, off));
  float *b = ball + g * (d + 1);
  if (lane < d) b[lane] = ck;
  if (lane == 0) b[d] = __builtin_sqrtf(r2) * (1.f + 0x1p-16f);
}

int grid_for(int64_t work, int threads) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + threads - 1) / threads, 65536));
}

}  // namespace

int64_t node_order_keys(int64_t n) {
  int64_t p2 = kSortSpan;
  while (p2 < n) p2 <<= 1;
  return p2;
}

hipError_t launch_node_order(const float *nodes, int64_t n, int d, uint64_t *keys, int32_t *perm, int32_t *rank,
                             float *xs, float *aabb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t p2 = node_order_keys(n);
  // The cloud box lives in the first 2d words of aabb (at least 2d floats
  // for n >= 1) until order_boxes_kernel overwrites them.
  uint32_t *box = reinterpret_cast<uint32_t *>(aabb);
  hipLaunchKernelGGL(cloud_box_init_kernel, dim3(1), dim3(64), 0, s, d, box);
  hipLaunchKernelGGL(cloud_box_kernel, dim3(std::min(grid_for(n, 256), kBoxBlocks)), dim3(256), 0, s, nodes, n, d,
                     box);
  hipLaunchKernelGGL(order_keys_kernel, dim3(grid_for(p2, 256)), dim3(256), 0, s, nodes, n, d, p2,
                     static_cast<const uint32_t *>(box), keys);
  const int spans = (int)(p2 / kSortSpan);
  hipLaunchKernelGGL(bitonic_local_kernel, dim3(spans), dim3(kSortThreads), 0, s, keys, (int64_t)0);
  for (int64_t k = 2 * kSortSpan; k <= p2; k <<= 1) {
    for (int64_t j = k / 2; j >= kSortSpan; j >>= 1)
      hipLaunchKernelGGL(bitonic_global_kernel, dim3(grid_for(p2 / 2, 256)), dim3(256), 0, s, keys, p2, k, j);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(spans), dim3(kSortThreads), 0, s, keys, k);
  }
  hipLaunchKernelGGL(order_apply_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, nodes, n, d, perm, rank,
                     xs);
  const int64_t groups = order_groups(n);
  hipLaunchKernelGGL(order_boxes_kernel, dim3((int)((groups + 3) / 4)), dim3(256), 0, s, xs, n, d, aabb,
                     aabb + groups * 2 * d);
  return hipGetLastError();
}

}  // namespace vg
