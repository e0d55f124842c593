// Generator adjacency from Voronoi vertex tuples (CSR), on the GPU.
//
// Two generators are neighbours when some vertex's (d+1)-tuple holds both:
// the vertex is equidistant to them and nearer to no other generator, so
// their bisector carries a face of both cells (the Delaunay edges of the
// tuple set).  Every ordered pair (a, b), a != b, of every tuple becomes the
// key (a << 32 | b); a radix sort and a unique pass leave each directed edge
// once, sorted by (a, b), which is already the CSR column array; per-row
// counts and an inclusive scan give the row offsets.
#include <hipcub/hipcub.hpp>

#include "vg_internal.h"

namespace vg {
namespace {

__global__ void tuple_check_kernel(const int32_t *__restrict__ sig, int64_t count, int64_t n,
                                   uint32_t *__restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count && (sig[t] < 0 || sig[t] >= n)) atomicOr(bad, 1u);
}

__global__ void tuple_pairs_kernel(const int32_t *__restrict__ sig, int64_t V, int L,
                                   uint64_t *__restrict__ keys) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (vertex, a)
  if (t >= V * L) return;
  const int64_t v = t / L;
  const int a = (int)(t - v * L);
  const int32_t *s = sig + v * L;
  const uint64_t hi = (uint64_t)(uint32_t)s[a] << 32;
  uint64_t *out = keys + t * (L - 1);
  int q = 0;
  for (int b = 0; b < L; ++b)
    if (b != a) out[q++] = hi | (uint32_t)s[b];
}

__global__ void csr_fill_kernel(const uint64_t *__restrict__ keys, int64_t nnz,
                                int32_t *__restrict__ nbr, unsigned long long *__restrict__ counts) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const uint64_t k = keys[p];
  nbr[p] = (int32_t)(uint32_t)(k & 0xffffffffu);
  atomicAdd(&counts[(k >> 32) + 1], 1ull);
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int tuple_neighbors(int d, int64_t n_nodes, int64_t n_tuples, const int32_t *sigma,
                    int64_t *offsets, int32_t *nbr, int64_t nbr_capacity, int64_t *nnz_out,
                    hipStream_t s, std::string &err) {
  const int L = d + 1;
  const int64_t P = n_tuples * L * (L - 1);
  if (P >= (int64_t(1) << 31)) {
    err = "more than 2^31 tuple pairs";
    return VG_EUNSUPPORTED;
  }
  int bits = 32;  // key bits: 32 for b, enough above them for a < n_nodes
  while (bits < 64 && (int64_t(1) << (bits - 32)) < n_nodes) ++bits;
  uint64_t *ka = nullptr, *kb = nullptr;
  unsigned long long *counts = nullptr;
  int64_t *dn = nullptr;
  uint32_t *bad = nullptr;
  void *tmp = nullptr;
  auto done = [&](int rc, const char *msg) {
    if (msg) err = msg;
    for (void *p : {(void *)ka, (void *)kb, (void *)counts, (void *)dn, (void *)bad, tmp})
      if (p) (void)hipFree(p);
    return rc;
  };
  auto hip = [&](hipError_t e) { return e == hipSuccess ? VG_OK : done(VG_EDEVICE, hipGetErrorString(e)); };
  if ((P > 0 && (hipMalloc(&ka, (size_t)P * 8) != hipSuccess || hipMalloc(&kb, (size_t)P * 8) != hipSuccess)) ||
      hipMalloc(&dn, 8) != hipSuccess || hipMalloc(&bad, 4) != hipSuccess ||
      hipMalloc(&counts, (size_t)(n_nodes + 1) * 8) != hipSuccess)
    return done(VG_ENOMEM, "neighbour list scratch allocation failed");

  // every tuple entry must be a node index
  int rc = hip(fill_u32(bad, 0u, 1, s));
  if (rc) return rc;
  if (n_tuples > 0) {
    hipLaunchKernelGGL(tuple_check_kernel, dim3(blocks(n_tuples * L)), dim3(256), 0, s, sigma,
                       n_tuples * L, n_nodes, bad);
    if ((rc = hip(hipGetLastError()))) return rc;
  }
  uint32_t hbad = 0;
  if ((rc = hip(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s)))) return rc;
  if ((rc = hip(hipStreamSynchronize(s)))) return rc;
  if (hbad) return done(VG_EINVAL, "sigma holds an entry outside [0, n_nodes)");

  // directed pairs, sorted and made unique
  int64_t nnz = 0;
  size_t b1 = 0, b2 = 0, b3 = 0;
  if (P > 0) {
    hipLaunchKernelGGL(tuple_pairs_kernel, dim3(blocks(n_tuples * L)), dim3(256), 0, s, sigma, n_tuples, L, ka);
    if ((rc = hip(hipGetLastError()))) return rc;
    if ((rc = hip(hipcub::DeviceRadixSort::SortKeys(nullptr, b1, ka, kb, (int)P, 0, bits, s)))) return rc;
    if ((rc = hip(hipcub::DeviceSelect::Unique(nullptr, b2, kb, ka, dn, (int)P, s)))) return rc;
  }
  if ((rc = hip(hipcub::DeviceScan::InclusiveSum(nullptr, b3, counts, (unsigned long long *)offsets,
                                                 (int)n_nodes + 1, s))))
    return rc;
  if (hipMalloc(&tmp, std::max<size_t>({b1, b2, b3, 16})) != hipSuccess)
    return done(VG_ENOMEM, "sort scratch allocation failed");
  if (P > 0) {
    if ((rc = hip(hipcub::DeviceRadixSort::SortKeys(tmp, b1, ka, kb, (int)P, 0, bits, s)))) return rc;
    if ((rc = hip(hipcub::DeviceSelect::Unique(tmp, b2, kb, ka, dn, (int)P, s)))) return rc;
    if ((rc = hip(hipMemcpyAsync(&nnz, dn, 8, hipMemcpyDeviceToHost, s)))) return rc;
    if ((rc = hip(hipStreamSynchronize(s)))) return rc;
  }
  *nnz_out = nnz;
  if (!offsets && !nbr) return done(VG_OK, nullptr);
  if (!offsets || !nbr) return done(VG_EINVAL, "offsets and nbr must both be set or both be NULL");
  if (nnz > nbr_capacity) return done(VG_EINVAL, "nbr_capacity is below the number of neighbour pairs");

  // CSR: columns are the sorted unique keys' low words; rows from counts
  if ((rc = hip(fill_u32(reinterpret_cast<uint32_t *>(counts), 0u, 2 * (n_nodes + 1), s)))) return rc;
  if (nnz > 0) {
    hipLaunchKernelGGL(csr_fill_kernel, dim3(blocks(nnz)), dim3(256), 0, s, ka, nnz, nbr, counts);
    if ((rc = hip(hipGetLastError()))) return rc;
  }
  if ((rc = hip(hipcub::DeviceScan::InclusiveSum(tmp, b3, counts, (unsigned long long *)offsets,
                                                 (int)n_nodes + 1, s))))
    return rc;
  if ((rc = hip(hipStreamSynchronize(s)))) return rc;
  return done(VG_OK, nullptr);
}

}  // namespace vg
