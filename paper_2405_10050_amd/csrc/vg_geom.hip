// FP64 geometry of the exhaustive search (Sec. 2.1, Algorithm 2), one thread
// per item:
//   * SearchDirection(sigma, eta): unit vector orthogonal to the affine span
//     of X_eta pointing away from the omitted generator; built as the
//     normalised negative of the component of (x_omit - x_eta0) orthogonal
//     to span{x_j - x_eta0}, by Gram-Schmidt applied twice;
//   * the vertex of sigma: the point equidistant to its d+1 generators, from
//     2 (x_b - x_a).y = |x_b - x_a|^2 (y = v - x_a), Gaussian elimination
//     with partial pivoting;
//   * on the diagram clipped to the unit cube, keys also hold faces x_k = s
//     (code face_base + 2k + s, after the generators): a kept face adds e_k
//     to the span the direction is orthogonal to, a dropped face makes the
//     direction point into the cube (w = -+e_k in place of x_omit - x_eta0),
//     and a face of the vertex adds the row y_k = s - x_a,k to the solve;
//   * the Descent projection (Algorithm 2): a random direction with its
//     component in the span of X_sigma removed;
//   * on the periodic diagram, key entries are images x_i + k (codes
//     i S + c(k)) taken exactly in FP64; rays run over the scanned images,
//     each new vertex's ball is checked to lie inside the scanned layer, and
//     its key is translated to the normal form (first entry k = 0) before
//     its coordinates are solved, so they depend on the vertex alone.
#include "vg_internal.h"
#include "vg_explore.h"

namespace vg {
namespace {

// The points of a key: node rows, or exact images of the periodic diagram.
struct NodePts {
  const float *X;
  int d;
  __device__ double operator()(int32_t e, int k) const { return (double)X[(int64_t)e * d + k]; }
};
struct ImagePts {
  Periodic P;
  int d;
  __device__ double operator()(int32_t e, int k) const { return image_coord(P, d, e, k); }
};

// Removes from w its components along span{e_k : faces among s} U
// {X[s_j] - X[s_0] : generators s_j, j > 0} (s_0 a generator; faces are
// the entries >= face_base), by Gram-Schmidt applied twice, faces first.
template <int DK, typename PT>
__device__ void orth_complement(const PT &pt, int d, const int32_t *s, int m, int32_t face_base, double *w) {
  // Q holds up to m-1 orthonormal vectors of the span
  double Q[DK - 1 > 0 ? DK - 1 : 1][DK];
  int q = 0;
  for (int j = 1; j < m; ++j) {
    if (s[j] < face_base) continue;
    // a face normal is orthogonal to the other faces' (distinct axes)
    const int k0 = (s[j] - face_base) / 2;
#pragma unroll
    for (int k = 0; k < DK; ++k) Q[q][k] = (k == k0) ? 1.0 : 0.0;
    ++q;
  }
  for (int j = 1; j < m; ++j) {
    if (s[j] >= face_base) continue;
    double e[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) e[k] = (k < d) ? pt(s[j], k) - pt(s[0], k) : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int a = 0; a < q; ++a) {
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < DK; ++k) c += e[k] * Q[a][k];
#pragma unroll
        for (int k = 0; k < DK; ++k) e[k] -= c * Q[a][k];
      }
    }
    double nr = 0.0;
#pragma unroll
    for (int k = 0; k < DK; ++k) nr += e[k] * e[k];
    nr = sqrt(nr);
    if (nr == 0.0) continue;
#pragma unroll
    for (int k = 0; k < DK; ++k) Q[q][k] = e[k] / nr;
    ++q;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int a = 0; a < q; ++a) {
      double c = 0.0;
#pragma unroll
      for (int k = 0; k < DK; ++k) c += w[k] * Q[a][k];
#pragma unroll
      for (int k = 0; k < DK; ++k) w[k] -= c * Q[a][k];
    }
  }
}

template <int DK, typename PT>
__device__ bool solve_vertex(const PT &pt, int d, const int32_t *s, int32_t face_base, double *v) {
  double A[DK][DK], b[DK], y[DK];
  for (int r = 0; r < DK; ++r) {
    b[r] = 0.0;
    for (int k = 0; k < DK; ++k) A[r][k] = 0.0;
  }
  for (int r = 0; r < d; ++r) {
    if (s[r + 1] >= face_base) {  // face x_k = side: y_k = side - x_a,k
      const int f = s[r + 1] - face_base;
      A[r][f / 2] = 1.0;
      b[r] = (double)(f % 2) - pt(s[0], f / 2);
      continue;
    }
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
      const double e = pt(s[r + 1], k) - pt(s[0], k);
      A[r][k] = 2.0 * e;
      acc += e * e;
    }
    b[r] = acc;
  }
  for (int c = 0; c < d; ++c) {
    int p = c;
    double pv = fabs(A[c][c]);
    for (int r = c + 1; r < d; ++r)
      if (fabs(A[r][c]) > pv) {
        pv = fabs(A[r][c]);
        p = r;
      }
    if (pv == 0.0) return false;
    if (p != c) {
      for (int k = 0; k < d; ++k) {
        const double tmp = A[c][k];
        A[c][k] = A[p][k];
        A[p][k] = tmp;
      }
      const double tmp = b[c];
      b[c] = b[p];
      b[p] = tmp;
    }
    for (int r = c + 1; r < d; ++r) {
      const double f = A[r][c] / A[c][c];
      for (int k = c; k < d; ++k) A[r][k] -= f * A[c][k];
      b[r] -= f * b[c];
    }
  }
  for (int c = d - 1; c >= 0; --c) {
    double acc = b[c];
    for (int k = c + 1; k < d; ++k) acc -= A[c][k] * y[k];
    y[c] = acc / A[c][c];
  }
  for (int k = 0; k < d; ++k) v[k] = pt(s[0], k) + y[k];
  for (int r = 1; r <= d; ++r)  // a vertex on a face lies on it exactly
    if (s[r] >= face_base) v[(s[r] - face_base) / 2] = (double)((s[r] - face_base) % 2);
  return true;
}

// Edge ray of a periodic item: the direction from the exact images; g and
// the exclusions are the kept images' rows in the scanned layer (sorted),
// and a kept image outside it marks the layer too thin.
template <int DK>
__device__ void edge_ray_periodic(const ExploreRays &a, int64_t it) {
  const int d = a.d;
  const int64_t v = a.item_v[it];
  const int o = a.item_o[it];
  const int32_t *sig = a.keys + v * (d + 1);
  int32_t eta[DK];
  int q = 0;
  for (int b = 0; b <= d; ++b)
    if (b != o) eta[q++] = sig[b];
  const ImagePts pt{a.per, d};
  double w[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) w[k] = (k < d) ? pt(sig[o], k) - pt(eta[0], k) : 0.0;
  orth_complement<DK>(pt, d, eta, d, INT32_MAX, w);
  double nr = 0.0;
#pragma unroll
  for (int k = 0; k < DK; ++k) nr += w[k] * w[k];
  nr = sqrt(nr);
  int32_t ex[DK];
  bool inside = true;
  for (int b = 0; b < d; ++b) {
    const int32_t e = eta[b];
    const int32_t r = (e >= 0 && (int64_t)e < a.per.n_codes) ? a.per.tix[e] : -1;
    inside = inside && r >= 0;
    ex[b] = r >= 0 ? r : INT32_MAX;
  }
  if (!inside) atomicOr(a.err, VSET_THIN);
  const bool good = nr > 0.0 && inside;
  a.gen[it] = inside ? ex[0] : 0;
  for (int b = 1; b < d; ++b) {  // insertion sort of the exclusions
    const int32_t x = ex[b];
    int c = b - 1;
    while (c >= 0 && ex[c] > x) {
      ex[c + 1] = ex[c];
      --c;
    }
    ex[c + 1] = x;
  }
  for (int b = 0; b < d; ++b) a.excl[it * d + b] = ex[b];
  for (int k = 0; k < d; ++k) {
    a.u64[it * d + k] = good ? -w[k] / nr : 0.0;
    a.o64[it * d + k] = a.coords[v * d + k];
  }
  a.ok[it] = good ? 1 : 0;
}

// New vertex of a periodic hit: the hit image's code joins the kept ones,
// the ball is checked against the layer in the frame of the ray, then the
// key is translated to its normal form and the vertex solved from it.
template <int DK>
__device__ void new_vertex_periodic(const ExploreRays &a, int64_t it) {
  const int d = a.d;
  const int32_t hit = a.idx[it];
  int32_t *key = a.new_keys + it * (d + 1);
  if (!a.ok[it]) {
    key[0] = -1;
    return;
  }
  if (hit < 0 || (int64_t)hit >= a.n_nodes) {  // no hit: the ray left the layer
    atomicOr(a.err, VSET_THIN);
    key[0] = -1;
    return;
  }
  const int32_t j = a.per.tkey[hit];
  const int32_t *sig = a.keys + a.item_v[it] * (d + 1);
  const int o = a.item_o[it];
  int32_t ks[DK + 1];
  int q = 0;
  bool placed = false;
  for (int b = 0; b <= d; ++b) {
    if (b == o) continue;
    if (!placed && j < sig[b]) {
      ks[q++] = j;
      placed = true;
    }
    ks[q++] = sig[b];
  }
  if (!placed) ks[q++] = j;
  const ImagePts pt{a.per, d};
  double v[DK];
  if (!solve_vertex<DK>(pt, d, ks, INT32_MAX, v)) {
    key[0] = -2;
    return;
  }
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double e = v[k] - pt(ks[0], k);
    r2 += e * e;
  }
  const double R = sqrt(r2);
  bool inside = true;
  for (int k = 0; k < d; ++k) inside = inside && v[k] - R > -a.per.w && v[k] + R < 1.0 + a.per.w;
  if (!inside) {
    atomicOr(a.err, VSET_THIN);
    key[0] = -1;
    return;
  }
  if (!periodic_canon(ks, d + 1, d, a.per.S)) {
    atomicOr(a.err, VSET_RANGE);
    key[0] = -1;
    return;
  }
  if (!solve_vertex<DK>(pt, d, ks, INT32_MAX, v)) {
    key[0] = -2;
    return;
  }
  for (int b = 0; b <= d; ++b) key[b] = ks[b];
  for (int k = 0; k < d; ++k) a.new_coords[it * d + k] = v[k];
}

// Edge rays of the frontier: item (vertex v, omitted position o).
template <int DK>
__global__ __launch_bounds__(128) void edge_rays_kernel(ExploreRays a) {
  const int64_t it = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (it >= a.m) return;
  if (a.per.S) {
    edge_ray_periodic<DK>(a, it);
    return;
  }
  const int d = a.d;
  const int64_t v = a.item_v[it];
  const int o = a.item_o[it];
  const int32_t *sig = a.keys + v * (d + 1);
  int32_t eta[DK];
  int q = 0;
  for (int b = 0; b <= d; ++b)
    if (b != o) eta[q++] = sig[b];
  const int32_t omit = sig[o];
  const int32_t fb = a.face_base;
  double w[DK];
  const float *x0 = a.nodes + (int64_t)eta[0] * d;
  if (omit < fb) {
    const float *xo = a.nodes + (int64_t)omit * d;
#pragma unroll
    for (int k = 0; k < DK; ++k) w[k] = (k < d) ? (double)xo[k] - (double)x0[k] : 0.0;
  } else {  // off the face x_k = side, into the cube: u_k of sign 1 - 2 side
    const int f = omit - fb;
#pragma unroll
    for (int k = 0; k < DK; ++k) w[k] = (k == f / 2) ? ((f % 2) ? 1.0 : -1.0) : 0.0;
  }
  orth_complement<DK>(NodePts{a.nodes, d}, d, eta, d, fb, w);
  double nr = 0.0;
#pragma unroll
  for (int k = 0; k < DK; ++k) nr += w[k] * w[k];
  nr = sqrt(nr);
  const bool good = nr > 0.0 && eta[0] < fb;
  for (int k = 0; k < d; ++k) {
    a.u64[it * d + k] = good ? -w[k] / nr : 0.0;
    a.o64[it * d + k] = a.coords[v * d + k];
  }
  a.gen[it] = eta[0];
  // the kept generators (sorted, first in the key), padded past the end
  for (int b = 0; b < d; ++b) a.excl[it * d + b] = eta[b] < fb ? eta[b] : INT32_MAX;
  a.ok[it] = good ? 1 : 0;
}

// New vertex of each hit: key sort(eta U {j}) and its FP64 coordinates.
template <int DK>
__global__ __launch_bounds__(128) void new_vertex_kernel(ExploreRays a) {
  const int64_t it = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (it >= a.m) return;
  if (a.per.S) {
    new_vertex_periodic<DK>(a, it);
    return;
  }
  const int d = a.d;
  const int32_t hit = a.idx[it];
  int32_t *key = a.new_keys + it * (d + 1);
  if (hit == -1 || !a.ok[it]) {
    key[0] = -1;
    return;
  }
  // a face hit -2-f (clipped rays only) is the constraint face_base + f
  const int32_t j = hit >= 0 ? hit : a.face_base + (-2 - hit);
  const int32_t *sig = a.keys + a.item_v[it] * (d + 1);
  const int o = a.item_o[it];
  int q = 0;
  bool placed = false;
  for (int b = 0; b <= d; ++b) {
    if (b == o) continue;
    if (!placed && j < sig[b]) {
      key[q++] = j;
      placed = true;
    }
    key[q++] = sig[b];
  }
  if (!placed) key[q++] = j;
  double v[DK];
  int32_t ks[DK + 1];
  for (int b = 0; b <= d; ++b) ks[b] = key[b];
  if (!solve_vertex<DK>(NodePts{a.nodes, d}, d, ks, a.face_base, v)) {
    key[0] = -2;  // singular: degenerate input
    return;
  }
  for (int k = 0; k < d; ++k) a.new_coords[it * d + k] = v[k];
}

template <int DK>
__global__ void descent_project_kernel(const float *X, int d, const int32_t *sig, int m,
                                       double *u, int *ok) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double w[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) w[k] = (k < d) ? u[k] : 0.0;
  orth_complement<DK>(NodePts{X, d}, d, sig, m, INT32_MAX, w);
  double nr = 0.0;
#pragma unroll
  for (int k = 0; k < DK; ++k) nr += w[k] * w[k];
  nr = sqrt(nr);
  for (int k = 0; k < d; ++k) u[k] = nr > 0.0 ? w[k] / nr : 0.0;
  *ok = nr > 0.0 ? 1 : 0;
}

__global__ void advance_kernel(double *r, const double *u, const double *t, int d, double sign) {
  const int k = threadIdx.x;
  if (k < d) r[k] += t[0] * sign * u[k];
}

template <int DK>
__global__ void solve_one_kernel(const float *X, int d, const int32_t *sig, Periodic per, double *v, int *ok) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t ks[DK + 1];
  for (int b = 0; b <= d; ++b) ks[b] = sig[b];
  double vv[DK];
  const bool good = per.S ? solve_vertex<DK>(ImagePts{per, d}, d, ks, INT32_MAX, vv)
                          : solve_vertex<DK>(NodePts{X, d}, d, ks, INT32_MAX, vv);
  for (int k = 0; k < d; ++k) v[k] = good ? vv[k] : 0.0;
  *ok = good ? 1 : 0;
}

// Empty-circumsphere check of new vertices (Sec. 2.2 incircle criterion):
// viol[it] = min over nodes r not in the key of (|r - v|^2 - rho^2) / rho^2,
// negative when a node lies strictly inside the vertex's sphere.
__global__ __launch_bounds__(256) void sphere_check_kernel(ExploreRays a, double *viol) {
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= a.m) return;
  const int d = a.d;
  const int32_t *key = a.new_keys + it * (d + 1);
  if (key[0] < 0) {
    viol[it] = 0.0;
    return;
  }
  const double *v = a.new_coords + it * d;
  const float *x0 = a.nodes + (int64_t)key[0] * d;
  double rho2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double e = (double)x0[k] - v[k];
    rho2 += e * e;
  }
  double worst = __builtin_inf();
  int kp = 0;
  for (int64_t r = 0; r < a.n_nodes; ++r) {
    if (kp <= d && key[kp] == (int32_t)r) {
      ++kp;
      continue;
    }
    const float *xr = a.nodes + r * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const double e = (double)xr[k] - v[k];
      s += e * e;
    }
    worst = fmin(worst, (s - rho2) / rho2);
  }
  viol[it] = worst;
}

}  // namespace

hipError_t launch_sphere_check(const ExploreRays &a, double *viol, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(sphere_check_kernel, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, a,
                     viol);
  return hipGetLastError();
}

#define VG_DK_DISPATCH(d, KERNEL, GRID, BLK, ...)                                     \
  do {                                                                                \
    if ((d) <= 4)                                                                     \
      hipLaunchKernelGGL(KERNEL<4>, GRID, BLK, 0, s, __VA_ARGS__);                    \
    else if ((d) <= 8)                                                                \
      hipLaunchKernelGGL(KERNEL<8>, GRID, BLK, 0, s, __VA_ARGS__);                    \
    else if ((d) <= 12)                                                               \
      hipLaunchKernelGGL(KERNEL<12>, GRID, BLK, 0, s, __VA_ARGS__);                   \
    else                                                                              \
      hipLaunchKernelGGL(KERNEL<16>, GRID, BLK, 0, s, __VA_ARGS__);                   \
  } while (0)

hipError_t launch_edge_rays(const ExploreRays &a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.m + 127) / 128)), blk(128);
  VG_DK_DISPATCH(a.d, edge_rays_kernel, grid, blk, a);
  return hipGetLastError();
}

hipError_t launch_new_vertices(const ExploreRays &a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.m + 127) / 128)), blk(128);
  VG_DK_DISPATCH(a.d, new_vertex_kernel, grid, blk, a);
  return hipGetLastError();
}

hipError_t launch_descent_project(const float *X, int d, const int32_t *sig, int m, double *u,
                                  int *ok, hipStream_t s) {
  VG_DK_DISPATCH(d, descent_project_kernel, dim3(1), dim3(64), X, d, sig, m, u, ok);
  return hipGetLastError();
}

hipError_t launch_advance(double *r, const double *u, const double *t, int d, double sign,
                          hipStream_t s) {
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, r, u, t, d, sign);
  return hipGetLastError();
}

hipError_t launch_solve_one(const float *X, int d, const int32_t *sig, const Periodic &per, double *v,
                            int *ok, hipStream_t s) {
  VG_DK_DISPATCH(d, solve_one_kernel, dim3(1), dim3(64), X, d, sig, per, v, ok);
  return hipGetLastError();
}

}  // namespace vg
