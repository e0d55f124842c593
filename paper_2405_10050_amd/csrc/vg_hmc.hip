// Heuristic Monte-Carlo integrals (Sec. 3.3) over the diagram clipped to the
// unit cube.
//
// Inputs: the clipped vertex set (keys of d+1 constraints: generators, then
// n + 2k + s for the face x_k = s), and the facet rows of the Monte-Carlo
// estimator of each cell i (facet_j, facet_area; a face is -2-(2k+s) there).
// For the facet (i, j):
//   V_ij = the vertices whose key holds both i and j (K_ij of them),
//   y_ij = their mean (the centroid of the facet),
//   F_ij = A_ij (d/(d+1) mean_k f(nu_k) + 1/(d+1) f(y_ij)),
// and the cell integral sums the pyramid rule over each facet with apex x_i:
//   cell_i   = sum_j h_ij/d (d/(d+1) F_ij + 1/(d+1) A_ij f(x_i)),
//   volume_i = sum_j h_ij A_ij / d,
// with h_ij the distance of x_i to the facet's hyperplane (|x_j - x_i|/2, or
// x_i,k / 1 - x_i,k for a face).
//
// Layout: each cell's vertex list is a CSR built by a stable radix sort of
// the (generator, vertex) pairs, so it is in vertex order.  One workgroup per
// cell; each thread owns facet rows and walks the cell's vertex list (the
// same key for every thread at a time), testing whether the key holds its
// row's j.  Sums run in vertex order and the cell's reduction is a fixed
// tree, so results are bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include "vg_internal.h"

namespace vg {
namespace {

constexpr int HT = 256;

// Pair (key entry, vertex) of every entry of every key; faces and invalid
// entries go to the bucket n (past the last cell).
__global__ void cell_pairs_kernel(const int32_t *__restrict__ sig, int64_t V, int L, int64_t n, int d,
                                  int32_t *__restrict__ keys, int32_t *__restrict__ vals, uint32_t *bad) {
  const int64_t t = (int64_t)blockIdx.x * HT + threadIdx.x;
  if (t >= V * L) return;
  const int32_t s = sig[t];
  if (s < 0 || (int64_t)s >= n + 2 * d) atomicOr(bad, 1u);
  keys[t] = (s >= 0 && s < n) ? s : (int32_t)n;
  vals[t] = (int32_t)(t / L);
}

// offs[a] = first position of key a in the sorted keys (a in [0, n]).
__global__ void csr_bounds_kernel(const int32_t *__restrict__ keys, int64_t P, int64_t n, int64_t *__restrict__ offs) {
  const int64_t a = (int64_t)blockIdx.x * HT + threadIdx.x;
  if (a > n) return;
  int64_t lo = 0, hi = P;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (keys[mid] < a)
      lo = mid + 1;
    else
      hi = mid;
  }
  offs[a] = lo;
}

struct HmcArgs {
  int d;
  int64_t n;
  const float *nodes;
  const int32_t *sig;     // [V][d+1]
  const double *coords;   // [V][d] (centroid pass)
  const float *fv;        // [V] f at the vertices (integral pass)
  const int64_t *offs;    // [n+1] cell vertex lists
  const int32_t *verts;
  int R;
  const int32_t *facet_j;
  const float *facet_area;
  const int32_t *facet_count;
  const float *fc;        // [n][R] f at the centroids
  const float *fx;        // [n] f at the generators
  float *centroid;        // [n][R][d]
  int32_t *kcount;        // [n][R]
  float *F;               // [n][R]
  float *cell;            // [n]
  float *volume;          // [n]
  uint32_t *bad;          // bit 0: bad input, bit 1: a facet with no vertex
};

__device__ __forceinline__ int32_t facet_code(int32_t j, int64_t n) {
  return j >= 0 ? j : (int32_t)(n + (-2 - j));
}

template <int DK, bool INTEGRALS>
__global__ __launch_bounds__(HT) void hmc_rows_kernel(HmcArgs a) {
  const int64_t i = blockIdx.x;
  const int d = a.d, L = d + 1;
  const int cnt = min(a.facet_count[i], a.R);
  const int64_t v0 = a.offs[i], v1 = a.offs[i + 1];
  double part_vol = 0.0, part_cell = 0.0;
  for (int r = threadIdx.x; r < cnt; r += HT) {
    const int64_t row = i * a.R + r;
    const int32_t j = a.facet_j[row];
    const int32_t code = facet_code(j, a.n);
    if (!(j >= 0 ? (int64_t)j < a.n : (j <= -2 && -2 - j < 2 * d))) {
      atomicOr(a.bad, 1u);
      continue;
    }
    int K = 0;
    double acc[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) acc[k] = 0.0;
    for (int64_t p = v0; p < v1; ++p) {
      const int32_t v = a.verts[p];
      const int32_t *key = a.sig + (int64_t)v * L;
      bool has = false;
      for (int q = 0; q < L; ++q) has |= key[q] == code;
      if (!has) continue;
      ++K;
      if (INTEGRALS) {
        acc[0] += (double)a.fv[v];
      } else {
#pragma unroll
        for (int k = 0; k < DK; ++k)
          if (k < d) acc[k] += a.coords[(int64_t)v * d + k];
      }
    }
    if (K == 0) atomicOr(a.bad, 2u);
    if (!INTEGRALS) {
      for (int k = 0; k < d; ++k) a.centroid[row * d + k] = K ? (float)(acc[k] / K) : 0.f;
      a.kcount[row] = K;
      continue;
    }
    const double A = (double)a.facet_area[row];
    const double w1 = (double)d / (d + 1), w0 = 1.0 / (d + 1);
    const double Fij = K ? A * (w1 * (acc[0] / K) + w0 * (double)a.fc[row]) : 0.0;
    a.F[row] = (float)Fij;
    const float *xi = a.nodes + i * d;
    double h;
    if (code < a.n) {
      const float *xj = a.nodes + (int64_t)code * d;
      double s2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double e = (double)xj[k] - (double)xi[k];
        s2 += e * e;
      }
      h = 0.5 * sqrt(s2);
    } else {
      const int f = (int)(code - a.n);
      h = (f % 2) ? 1.0 - (double)xi[f / 2] : (double)xi[f / 2];
    }
    part_vol += h * A / d;
    part_cell += h / d * (w1 * Fij + w0 * A * (double)a.fx[i]);
  }
  if (!INTEGRALS) return;
  __shared__ double sv[HT], sc[HT];
  sv[threadIdx.x] = part_vol;
  sc[threadIdx.x] = part_cell;
  __syncthreads();
  for (int w = HT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sv[threadIdx.x] += sv[threadIdx.x + w];
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.volume[i] = (float)sv[0];
    a.cell[i] = (float)sc[0];
  }
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + HT - 1) / HT); }

}  // namespace

// Builds the cell vertex lists in temporary device memory, runs the row pass
// and frees them; synchronises the stream.  Returns VG_OK, VG_EINVAL (bad
// keys or facet codes, or a facet row whose pair no vertex holds) or a
// device error.
int hmc_run(bool integrals, int d, int64_t n, const float *nodes, int64_t V, const int32_t *sigma,
            const double *coords, const float *fv, int R, const int32_t *facet_j, const float *facet_area,
            const int32_t *facet_count, const float *fc, const float *fx, float *centroid, int32_t *kcount,
            float *F, float *cell, float *volume, hipStream_t s, std::string &err) {
  const int L = d + 1;
  const int64_t P = V * L;
  if (P >= (int64_t(1) << 31)) {
    err = "more than 2^31 vertex key entries";
    return VG_EUNSUPPORTED;
  }
  int32_t *ka = nullptr, *kb = nullptr, *va = nullptr, *vb = nullptr;
  int64_t *offs = nullptr;
  uint32_t *bad = nullptr;
  void *tmp = nullptr;
  auto done = [&](int rc, const char *msg) {
    if (msg) err = msg;
    for (void *p : {(void *)ka, (void *)kb, (void *)va, (void *)vb, (void *)offs, (void *)bad, tmp})
      if (p) (void)hipFree(p);
    return rc;
  };
  const size_t pb = (size_t)std::max<int64_t>(P, 1) * 4;
  if (hipMalloc(&ka, pb) != hipSuccess || hipMalloc(&kb, pb) != hipSuccess || hipMalloc(&va, pb) != hipSuccess ||
      hipMalloc(&vb, pb) != hipSuccess || hipMalloc(&offs, (size_t)(n + 1) * 8) != hipSuccess ||
      hipMalloc(&bad, 4) != hipSuccess)
    return done(VG_ENOMEM, "HMC scratch allocation failed");
  auto hip = [&](hipError_t e) { return e == hipSuccess ? VG_OK : done(VG_EDEVICE, hipGetErrorString(e)); };
  int rc = hip(fill_u32(bad, 0u, 1, s));
  if (rc) return rc;
  if (P > 0) hipLaunchKernelGGL(cell_pairs_kernel, dim3(blocks_of(P)), dim3(HT), 0, s, sigma, V, L, n, d, ka, va, bad);
  rc = hip(hipGetLastError());
  if (rc) return rc;
  int end_bit = 1;
  while (end_bit < 32 && (int64_t(1) << end_bit) <= n) ++end_bit;
  hipcub::DoubleBuffer<int32_t> dk(ka, kb), dv(va, vb);
  size_t tb = 0;
  rc = hip(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, dk, dv, (int)P, 0, end_bit, s));
  if (rc) return rc;
  if (hipMalloc(&tmp, std::max<size_t>(tb, 16)) != hipSuccess) return done(VG_ENOMEM, "HMC sort scratch allocation failed");
  rc = hip(hipcub::DeviceRadixSort::SortPairs(tmp, tb, dk, dv, (int)P, 0, end_bit, s));
  if (rc) return rc;
  hipLaunchKernelGGL(csr_bounds_kernel, dim3(blocks_of(n + 1)), dim3(HT), 0, s, dk.Current(), P, n, offs);
  rc = hip(hipGetLastError());
  if (rc) return rc;
  HmcArgs a{};
  a.d = d;
  a.n = n;
  a.nodes = nodes;
  a.sig = sigma;
  a.coords = coords;
  a.fv = fv;
  a.offs = offs;
  a.verts = dv.Current();
  a.R = R;
  a.facet_j = facet_j;
  a.facet_area = facet_area;
  a.facet_count = facet_count;
  a.fc = fc;
  a.fx = fx;
  a.centroid = centroid;
  a.kcount = kcount;
  a.F = F;
  a.cell = cell;
  a.volume = volume;
  a.bad = bad;
  const dim3 grid((unsigned)n), blk(HT);
  if (integrals) {
    hipLaunchKernelGGL((hmc_rows_kernel<1, true>), grid, blk, 0, s, a);
  } else if (d <= 4) {
    hipLaunchKernelGGL((hmc_rows_kernel<4, false>), grid, blk, 0, s, a);
  } else if (d <= 8) {
    hipLaunchKernelGGL((hmc_rows_kernel<8, false>), grid, blk, 0, s, a);
  } else {
    hipLaunchKernelGGL((hmc_rows_kernel<16, false>), grid, blk, 0, s, a);
  }
  rc = hip(hipGetLastError());
  if (rc) return rc;
  uint32_t bh = 0;
  rc = hip(hipMemcpyAsync(&bh, bad, 4, hipMemcpyDeviceToHost, s));
  if (rc) return rc;
  rc = hip(hipStreamSynchronize(s));
  if (rc) return rc;
  if (bh & 1u) return done(VG_EINVAL, "vertex keys or facet codes out of range");
  if (bh & 2u) return done(VG_EINVAL, "a facet row names a pair that no vertex holds (mesh and facets disagree)");
  return done(VG_OK, nullptr);
}

}  // namespace vg
