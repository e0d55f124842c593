// Scan order of the nodes for the Monte-Carlo cell scan.
//
// The cell scan visits every node for every ray of a cell (Algorithm 3 over
// eq. (t)), but a 32-node block whose largest |r~| = 1/|r - x_i| is below
// every lane's current second-best value cannot change any ray's top two and
// is skipped (the skip is exact: the result is the one of the full scan).
// Such blocks are frequent only when the nodes of a block lie close to each
// other, so the scan runs over a copy of the nodes sorted along a Morton
// (Z-order) curve of their first min(3, d) coordinates, and each cell starts
// at its own place in that order and works outwards: the blocks near x_i,
// which hold the rays' winners, come first and raise the second-best values
// before the far blocks are reached.
//
// The pass also records the bounding box of every 128 consecutive nodes of
// the sorted copy, from which the scan bounds whole chunks of nodes.
//
// The order is a pure function of the coordinates: the sort key is
// (Morton code << 32) | node index, unique per node, so any correct sort gives
// the same permutation.  Sort: bitonic over the next power of two of n (pads
// are all-ones keys), in LDS for spans up to 1024 and in global memory above;
// plain kernels only, so a caller may capture the pass in a hipGraph.
#include "vg_internal.h"

namespace vg {
namespace {

constexpr int kSortSpan = 1024;  // keys sorted in LDS by one workgroup
constexpr int kSortThreads = kSortSpan / 2;

// Morton code of the first min(3, d) coordinates (16 bits in all; each
// coordinate of the unit cube quantised to 16 / min(3, d) bits, values
// outside [0, 1) and NaN clamped).
__device__ __forceinline__ uint32_t morton_key(const float *x, int d) {
  const int m = d < 3 ? d : 3;
  const int bits = 16 / m;
  const float scale = (float)(1 << bits);
  uint32_t q[3] = {0u, 0u, 0u};
  for (int k = 0; k < m; ++k) {
    const float v = x[k] * scale;
    q[k] = v >= 1.f ? (v < scale ? (uint32_t)v : (uint32_t)((1 << bits) - 1)) : 0u;
  }
  uint32_t code = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int k = 0; k < m; ++k) code = (code << 1) | ((q[k] >> b) & 1u);
  return code;
}

__global__ void order_keys_kernel(const float *__restrict__ nodes, int64_t n, int d, int64_t p2,
                                  uint64_t *__restrict__ keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p2; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = i < n ? ((uint64_t)morton_key(nodes + i * d, d) << 32) | (uint64_t)i : ~0ull;
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

// Bounding box of each kOrderGroup consecutive nodes of xs: one wave per
// group, two nodes per lane, then a reduction over the lanes per coordinate.
__global__ __launch_bounds__(256) void order_boxes_kernel(const float *__restrict__ xs, int64_t n, int d,
                                                          float *__restrict__ aabb) {
  const int lane = threadIdx.x & 63;
  const int64_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ng = (n + kOrderGroup - 1) / kOrderGroup;
  if (g >= ng) return;
  for (int k = 0; k < d; ++k) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int e = lane; e < kOrderGroup; e += 64) {
      const int64_t p = g * kOrderGroup + e;
      if (p < n) {
        const float v = xs[p * d + k];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      aabb[g * 2 * d + k] = lo;
      aabb[g * 2 * d + d + k] = hi;
    }
  }
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
  hipLaunchKernelGGL(order_keys_kernel, dim3(grid_for(p2, 256)), dim3(256), 0, s, nodes, n, d, p2, keys);
  const int spans = (int)(p2 / kSortSpan);
  hipLaunchKernelGGL(bitonic_local_kernel, dim3(spans), dim3(kSortThreads), 0, s, keys, (int64_t)0);
  for (int64_t k = 2 * kSortSpan; k <= p2; k <<= 1) {
    for (int64_t j = k / 2; j >= kSortSpan; j >>= 1)
      hipLaunchKernelGGL(bitonic_global_kernel, dim3(grid_for(p2 / 2, 256)), dim3(256), 0, s, keys, p2, k, j);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(spans), dim3(kSortThreads), 0, s, keys, k);
  }
  hipLaunchKernelGGL(order_apply_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, keys, nodes, n, d, perm, rank,
                     xs);
  const int64_t groups = (n + kOrderGroup - 1) / kOrderGroup;
  hipLaunchKernelGGL(order_boxes_kernel, dim3((int)((groups + 3) / 4)), dim3(256), 0, s, xs, n, d, aabb);
  return hipGetLastError();
}

}  // namespace vg
