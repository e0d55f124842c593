// Monte-Carlo volume / interface-area estimators of Sec. 3.1 (Algorithm 3),
// the integrals of a function f over cells and facets, and the adjoint of
// the f = 1 estimators, on top of the per-ray RayCast results.
//
// Forward, one workgroup per cell (its rays are contiguous):
//   volume   = S/(d n)     sum l^d
//   energy2  = S/((d+2) n) sum l^{d+2}            (second moment about x_i)
//   area_ij  = S/n sum_{k: j_k = j} l^{d-1}/|n_ij.u|
// For a node j the ray meets the bisector at distance h = |x_j - x_i|/2 from
// x_i, so l |n_ij.u| = h and the area term equals 2 l^d / |x_j - x_i|; for a
// cube face at distance h it is l^d / h.  This form needs no division by the
// (possibly tiny) cosine.  Facets: the (j, ray) keys of the cell are sorted
// in LDS (bitonic), runs of equal j are summed in ray order, so every sum has
// a fixed order and the result is bitwise reproducible.  Integrals of f:
//   F_V[i]  = S/(n m) sum_k l^d sum_s f(x_i + t_s l u) t_s^{d-1}
//   F(i, j) = S/n sum_{k: j_k = j} f(x_i + l u) * (area term of ray k)
// with f evaluated by the caller at the points of sample_points_kernel.
//
// Adjoint, with the directions frozen (not in the paper):
//   node winner j, D = x_j - x_i, t = |D|^2/(2 u.D):
//     dt/dD = (D - t u)/(u.D) = 2 t (D - t u)/|D|^2,
//     dt/dx_j = dt/dD, dt/dx_i = -dt/dD;
//     the area term w = 2 l^d/|D| also has dw/dD|_l = -2 l^d D/|D|^3;
//   cube face x_k = s, h = |s - x_ik|: dt/dx_ik = -1/u_k, w = l^d/h with
//     dw/dx_ik|_l = l^d/h^2 * (s ? 1 : -1).
// The part landing on x_i is summed in the cell's workgroup.  The part
// landing on the winner x_j is scattered with 64-bit integer atomics in a
// per-node fixed-point scale chosen from that node's largest incoming
// magnitude and count (integer addition is associative, so the result does
// not depend on the order of the atomics).
#include <algorithm>

#include "vg_internal.h"
#include "vg_philox.h"

namespace vg {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ uint64_t facet_key(int32_t j, int ray) {
  return ((uint64_t)((uint32_t)j ^ 0x80000000u) << 32) | (uint32_t)ray;
}
__device__ __forceinline__ int32_t key_j(uint64_t k) {
  return (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
}

__device__ __forceinline__ float powi(float x, int p) {
  float r = 1.f;
  for (int q = 0; q < p; ++q) r *= x;
  return r;
}

// Deterministic block sum of one float per thread (tree in LDS).
__device__ float block_sum(float v, float *red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

__device__ void bitonic_sort(uint64_t *keys, int P) {
  const int tid = threadIdx.x;
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = tid; i < (P >> 1); i += NT) {
        const int lo = (i / stride) * 2 * stride + (i % stride);
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = keys[lo], b = keys[hi];
        if ((a > b) == asc) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
    }
  }
  __syncthreads();
}

// The terms of ray k of `cell`: l^d, l^{d+2}, the volume integrand of f
// (sum_s f(x_i + t_s l u) t_s^{d-1} l^d) and the area weight, computed as
// 2 l^d / |x_j - x_i| (= l^{d-1} / |n.u| at the bisector) or l^d / h for a
// cube face at distance h; its facet key (j, k).
template <int DK>
__device__ __forceinline__ void ray_terms(const AccumArgs &a, int64_t cell, const float (&xi)[DK], int k,
                                          float &ld, float &le, float &lf, float &wa, uint64_t &key) {
  const int d = a.d, R = a.R, M1 = a.m + 1;
  const int64_t gid = cell * R + k;
  const float l = a.t[gid];
  const int32_t j = a.idx[gid];
  ld = powi(l, d);
  le = ld * l * l;
  lf = 0.f;
  if (a.fvals && a.m > 0) {
    float g = 0.f;
    for (int q = 0; q < a.m; ++q) g += a.fvals[gid * M1 + 1 + q] * powi(a.tsamp[gid * a.m + q], d - 1);
    lf = g * ld;
  }
  wa = 0.f;
  if (j >= 0) {
    const float *xj = a.nodes + (int64_t)j * d;
    float n2 = 0.f;
#pragma unroll
    for (int q = 0; q < DK; ++q) {
      if (q < d) {
        const float e = xj[q] - xi[q];
        n2 = __builtin_fmaf(e, e, n2);
      }
    }
    wa = 2.f * ld / sqrtf(n2);
  } else if (j <= -2) {
    const int face = -2 - j, kk = face >> 1;
    float xk = 0.f;
#pragma unroll
    for (int q = 0; q < DK; ++q)
      if (q == kk) xk = xi[q];
    const float h = (face & 1) ? 1.f - xk : xk;
    wa = ld / h;
  }
  key = facet_key(j, k);
}

template <int DK>
__global__ __launch_bounds__(NT) void accum_kernel(AccumArgs a) {
  // one 16-byte aligned dynamic block: keys [P] u64 | w [P] f32 | red [NT] f32 | seg [NT+1] i32
  extern __shared__ __align__(16) uint64_t smem[];
  const int R = a.R;
  int P = 1;
  while (P < R) P <<= 1;
  uint64_t *keys = smem;
  float *w = reinterpret_cast<float *>(keys + P);
  float *red = w + P;
  int32_t *seg = reinterpret_cast<int32_t *>(red + NT);

  const int tid = threadIdx.x;
  const int64_t cell = blockIdx.x;
  const int d = a.d;
  float xi[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) xi[k] = (k < d) ? a.nodes[cell * d + k] : 0.f;

  float pv = 0.f, pe = 0.f, pf = 0.f;
  const int M1 = a.m + 1;
  for (int k = tid; k < P; k += NT) {
    if (k < R) {
      float ld, le, lf, wa;
      uint64_t key;
      ray_terms<DK>(a, cell, xi, k, ld, le, lf, wa, key);
      pv += ld;
      pe += le;
      pf += lf;
      keys[k] = key;
      w[k] = wa;
    } else {
      keys[k] = ~0ull;
    }
  }
  const float sum_v = block_sum(pv, red);
  const float sum_e = block_sum(pe, red);
  const float sum_f = a.fint_volume ? block_sum(pf, red) : 0.f;  // uniform condition
  if (tid == 0) {
    if (a.volume) a.volume[cell] = a.sv * sum_v;
    if (a.energy2) a.energy2[cell] = a.se * sum_e;
    if (a.fint_volume) a.fint_volume[cell] = a.sf * sum_f;
  }
  if (!a.facet_j) return;

  bitonic_sort(keys, P);
  // heads of runs of equal j, counted per thread over a contiguous segment
  const int E = (P + NT - 1) / NT;
  const int p0 = tid * E, p1 = min(p0 + E, R);
  int nh = 0;
  for (int p = p0; p < p1; ++p)
    if (p == 0 || (keys[p] >> 32) != (keys[p - 1] >> 32)) ++nh;
  // inclusive scan of the head counts: within each wave by shuffles, then
  // the totals of the waves before it
  {
    __shared__ int wave_tot[NT / 64];
    const int lane = tid & 63, wave = tid >> 6;
    int v = nh;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(v, off);
      if (lane >= off) v += o;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    for (int w2 = 0; w2 < wave; ++w2) v += wave_tot[w2];
    seg[tid + 1] = v;
    if (tid == 0) seg[0] = 0;
    __syncthreads();
  }
  // run sums of the ray weights: the areas, then (weights times f at the
  // hit point) the facet integrals of f
  for (int pass = 0; pass < 2; ++pass) {
    float *out = pass == 0 ? a.facet_area : a.fint_facet;
    if (pass == 1) {
      if (!a.fint_facet) break;
      __syncthreads();
      for (int k = tid; k < R; k += NT) w[k] *= a.fvals[(cell * R + k) * M1];
      __syncthreads();
    }
    int slot = seg[tid];
    for (int p = p0; p < p1; ++p) {
      if (p == 0 || (keys[p] >> 32) != (keys[p - 1] >> 32)) {
        float s = 0.f;
        int q = p;
        while (q < R && (keys[q] >> 32) == (keys[p] >> 32)) {
          s += w[(uint32_t)keys[q]];
          ++q;
        }
        if (pass == 0) a.facet_j[cell * R + slot] = key_j(keys[p]);
        if (out) out[cell * R + slot] = a.sa * s;
        ++slot;
      }
    }
  }
  if (tid == 0) a.facet_count[cell] = seg[NT];
}

// The same for at most 64 rays per cell: one wave per cell (four cells per
// workgroup), each lane one ray.  The facet keys are sorted across the wave
// by a bitonic network of shuffles, runs of equal j are found against the
// neighbouring lane, and their weights summed by a segmented scan, so no
// LDS and no barrier is needed.  Sums run in a shuffle tree, so they agree
// with the workgroup kernel's to rounding.
__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Inclusive sums of v within runs that start at the lanes with head set.
__device__ __forceinline__ float segmented_scan(float v, bool head, int lane) {
  int f = head ? 1 : 0;
  for (int off = 1; off < 64; off <<= 1) {
    const float ov = __shfl_up(v, off);
    const int of = __shfl_up(f, off);
    if (lane >= off && !f) {
      v += ov;
      f = of;
    }
  }
  return v;
}

template <int DK>
__global__ __launch_bounds__(NT) void accum_wave_kernel(AccumArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t cell = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (cell >= a.n) return;  // the whole wave
  const int d = a.d, R = a.R, M1 = a.m + 1;
  float xi[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) xi[k] = (k < d) ? a.nodes[cell * d + k] : 0.f;
  float ld = 0.f, le = 0.f, lf = 0.f, wa = 0.f;
  uint64_t key = ~0ull;
  if (lane < R) ray_terms<DK>(a, cell, xi, lane, ld, le, lf, wa, key);
  const float sum_v = wave_sum(ld), sum_e = wave_sum(le), sum_f = wave_sum(lf);
  if (lane == 0) {
    if (a.volume) a.volume[cell] = a.sv * sum_v;
    if (a.energy2) a.energy2[cell] = a.se * sum_e;
    if (a.fint_volume) a.fint_volume[cell] = a.sf * sum_f;
  }
  if (!a.facet_j) return;
  // bitonic sort of the 64 keys, ascending
  for (int size = 2; size <= 64; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t other = __shfl_xor(key, stride);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const uint64_t lo = key < other ? key : other, hi = key < other ? other : key;
      key = (lower == up) ? lo : hi;
    }
  }
  const uint32_t hj = (uint32_t)(key >> 32);
  const uint32_t prev = __shfl_up(hj, 1);
  const uint32_t next = __shfl_down(hj, 1);
  const bool valid = lane < R;
  const bool head = valid && (lane == 0 || prev != hj);
  const bool tail = valid && (lane == R - 1 || next != hj);
  const unsigned long long heads = __ballot(head);
  const int slot = __popcll(heads & ((2ull << lane) - 1ull)) - 1;  // run of this lane
  const int ray = valid ? (int)(uint32_t)key : 0;
  for (int pass = 0; pass < 2; ++pass) {
    float *out = pass == 0 ? a.facet_area : a.fint_facet;
    if (pass == 1 && !a.fint_facet) break;
    float w = __shfl(wa, ray);  // the weight of the ray now at this lane
    if (pass == 1) w *= valid ? a.fvals[(cell * R + ray) * M1] : 0.f;
    const float run = segmented_scan(valid ? w : 0.f, head, lane);
    if (tail) {
      if (pass == 0) a.facet_j[cell * R + slot] = key_j(key);
      if (out) out[cell * R + slot] = a.sa * run;
    }
  }
  if (lane == 0) a.facet_count[cell] = __popcll(heads);
}

// Algorithm 3's sample points of every ray: the hit point, then the interior
// points at the draws t_s (x_i + t_s l u, the same point as (1-t) x_i + t r).
template <int DK>
__global__ __launch_bounds__(NT) void sample_points_kernel(const float *__restrict__ nodes, int64_t n, int d,
                                                           int R, const float *__restrict__ dirs,
                                                           const float *__restrict__ t, int m,
                                                           const float *__restrict__ tsamp,
                                                           float *__restrict__ points) {
  const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (gid >= n * R) return;
  const int64_t cell = gid / R;
  const float l = t[gid];
  float xi[DK], u[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    xi[k] = k < d ? nodes[cell * d + k] : 0.f;
    u[k] = k < d ? dirs[gid * d + k] : 0.f;
  }
  float *out = points + gid * (m + 1) * d;
  for (int s = 0; s <= m; ++s) {
    const float tl = s == 0 ? l : tsamp[gid * m + s - 1] * l;
#pragma unroll
    for (int k = 0; k < DK; ++k)
      if (k < d) out[s * d + k] = __builtin_fmaf(tl, u[k], xi[k]);
  }
}

// ----------------------------------------------------------------- adjoint
// Per-cell tables of the winners of a round of rays, shared by the adjoint
// kernels: a cell's rays meet far fewer winners than there are rays (about
// 180 per 1024 rays of the d=10 mixture), so their global atomics are first
// combined per winner in LDS.  Rays go in rounds of kScatterRays; a round's
// winners fill at most half of the open-addressing table, so a probe always
// ends.
constexpr int kScatterRays = 1024;
constexpr int kScatterSlots = 2 * kScatterRays;
constexpr int kScatterLog2 = 11;
static_assert((1 << kScatterLog2) == kScatterSlots, "table size");

// Slot of winner j (inserted if new; a new slot is appended to used).
__device__ __forceinline__ int winner_slot(int32_t *key, int32_t *used, int *n_used, int32_t j) {
  uint32_t h = ((uint32_t)j * 2654435761u) >> (32 - kScatterLog2);
  for (;;) {
    const int32_t old = atomicCAS(&key[h], -1, j);
    if (old == -1) {
      used[atomicAdd(n_used, 1)] = (int32_t)h;
      return (int)h;
    }
    if (old == j) return (int)h;
    h = (h + 1) & (kScatterSlots - 1);
  }
}

template <int DK>
__global__ __launch_bounds__(NT) void backward_rays_kernel(BackwardArgs a) {
  __shared__ float red[NT];
  __shared__ int32_t key[kScatterSlots];  // winner of a slot, -1: free
  __shared__ uint32_t wmax[kScatterSlots];  // largest |record| (float bits) per winner
  __shared__ uint32_t wcnt[kScatterSlots];  // records per winner
  __shared__ int32_t used[kScatterRays];
  __shared__ int n_used;
  const int tid = threadIdx.x;
  for (int sl = tid; sl < kScatterSlots; sl += NT) {
    key[sl] = -1;
    wmax[sl] = 0u;
    wcnt[sl] = 0u;
  }
  if (tid == 0) n_used = 0;
  __syncthreads();
  const int64_t cell = blockIdx.x;
  const int d = a.d, R = a.R;
  float xi[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) xi[k] = (k < d) ? a.nodes[cell * d + k] : 0.f;
  const float gv = a.gv ? a.gv[cell] : 0.f;
  const float ge = a.ge ? a.ge[cell] : 0.f;
  const int nf = a.facet_count ? a.facet_count[cell] : 0;
  const int32_t *fj = a.facet_j ? a.facet_j + cell * R : nullptr;

  float own[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) own[k] = 0.f;

  for (int r0 = 0; r0 < R; r0 += kScatterRays) {
    const int r1 = min(R, r0 + kScatterRays);
    for (int kr = r0 + tid; kr < r1; kr += NT) {
      const int64_t gid = cell * R + kr;
      const float l = a.t[gid];
      const int32_t j = a.idx[gid];
      const float ld1 = powi(l, d - 1);
      const float ld = ld1 * l;
      // upstream weight of the facet this ray contributes to
      float ga = 0.f;
      if (a.ga && fj) {
        int lo = 0, hi = nf - 1;
        while (lo <= hi) {  // facets sorted by j as signed int
          const int mid = (lo + hi) >> 1;
          const int32_t v = fj[mid];
          if (v == j) {
            ga = a.ga[cell * R + mid];
            break;
          }
          if (v < j)
            lo = mid + 1;
          else
            hi = mid - 1;
        }
      }
      float dl = gv * a.sv * (float)d * ld1 + ge * a.se * (float)(d + 2) * ld * l;
      float win[DK];
#pragma unroll
      for (int k = 0; k < DK; ++k) win[k] = 0.f;
      if (j >= 0) {
        const float *xj = a.nodes + (int64_t)j * d;
        float D[DK], n2 = 0.f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          D[k] = (k < d) ? xj[k] - xi[k] : 0.f;
          n2 = __builtin_fmaf(D[k], D[k], n2);
        }
        const float nD = sqrtf(n2);
        dl += ga * a.sa * 2.f * (float)d * ld1 / nD;
        const float c = dl * 2.f * l / n2;             // dl * dt/dD scale
        const float cw = -ga * a.sa * 2.f * ld / (n2 * nD);  // direct area term
        float uk[DK];
        cell_dir<DK>(a.dirs, a.seed, cell, R, kr, d, uk);
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          win[k] = c * (D[k] - l * uk[k]) + cw * D[k];
          own[k] -= win[k];
        }
      } else if (j <= -2) {
        const int face = -2 - j, kk = face >> 1;
        float xk = 0.f;
#pragma unroll
        for (int q = 0; q < DK; ++q)
          if (q == kk) xk = xi[q];
        float ud[DK];
        cell_dir<DK>(a.dirs, a.seed, cell, R, kr, d, ud);
        float uk = 0.f;
#pragma unroll
        for (int q = 0; q < DK; ++q)
          if (q == kk) uk = ud[q];
        const float h = (face & 1) ? 1.f - xk : xk;
        dl += ga * a.sa * (float)d * ld1 / h;
        const float gk = dl * (-1.f / uk) + ga * a.sa * ld / (h * h) * ((face & 1) ? 1.f : -1.f);
#pragma unroll
        for (int q = 0; q < DK; ++q)
          if (q == kk) own[q] += gk;
      }
      // record the contribution aimed at the winner
      a.rec_j[gid] = j >= 0 ? j : -1;
      if (j >= 0) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          if (k < d) {
            a.rec[gid * d + k] = win[k];
            m = fmaxf(m, fabsf(win[k]));
          }
        }
        // |record| >= 0, so its bits order like the value
        const int sl = winner_slot(key, used, &n_used, j);
        atomicMax(&wmax[sl], __float_as_uint(m));
        atomicAdd(&wcnt[sl], 1u);
      }
    }
    __syncthreads();
    // one global max and count per winner of the round (both exact in any order)
    const int nu = n_used;
    for (int e = tid; e < nu; e += NT) {
      const int sl = used[e];
      atomicMax(&a.maxabs[key[sl]], wmax[sl]);
      atomicAdd(&a.count[key[sl]], wcnt[sl]);
      key[sl] = -1;
      wmax[sl] = 0u;
      wcnt[sl] = 0u;
    }
    __syncthreads();
    if (tid == 0) n_used = 0;
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    if (k < d) {
      const float s = block_sum(own[k], red);
      if (tid == 0) a.own[cell * d + k] = s;
    }
  }
}

__device__ __forceinline__ int fixed_scale(uint32_t maxbits, uint32_t count) {
  const float m = __uint_as_float(maxbits);
  int e;
  frexpf(m, &e);  // m < 2^e
  int c = 0;
  while ((1u << c) < count && c < 31) ++c;  // count <= 2^c
  return 61 - c - e;
}

// Winner-side part of the adjoint, one workgroup per cell: the records of
// the cell's rays are summed per winner j in LDS, as fixed-point int64 at
// j's scale, then added to acc with one global atomic per (winner,
// coordinate) instead of one per (ray, coordinate).  Integer addition is
// associative, so neither the LDS nor the global order of the additions
// changes a bit of the result.

template <int DK>
__global__ __launch_bounds__(NT) void backward_scatter_kernel(BackwardArgs a) {
  constexpr int PER = kScatterRays / NT;  // rays per thread and round
  __shared__ int32_t key[kScatterSlots];  // winner of a slot, -1: free
  __shared__ unsigned long long val[kScatterSlots];
  __shared__ int32_t used[kScatterRays];  // slots taken in this round
  __shared__ int n_used;
  const int d = a.d, R = a.R, tid = threadIdx.x;
  const int64_t cell = blockIdx.x;
  for (int sl = tid; sl < kScatterSlots; sl += NT) {
    key[sl] = -1;
    val[sl] = 0ull;
  }
  if (tid == 0) n_used = 0;
  __syncthreads();
  for (int r0 = 0; r0 < R; r0 += kScatterRays) {
    int slot[PER], F[PER];
    float v[PER][DK];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int r = r0 + p * NT + tid;
      slot[p] = -1;
      F[p] = 0;
      if (r >= R) continue;
      const int64_t gid = cell * R + r;
      const int32_t j = a.rec_j[gid];
      if (j < 0) continue;
      const uint32_t mb = a.maxabs[j];
      if (mb == 0) continue;
      F[p] = fixed_scale(mb, a.count[j]);
#pragma unroll
      for (int k = 0; k < DK; ++k) v[p][k] = k < d ? a.rec[gid * d + k] : 0.f;
      slot[p] = winner_slot(key, used, &n_used, j);
    }
    __syncthreads();
    const int nu = n_used;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {  // uniform
#pragma unroll
        for (int p = 0; p < PER; ++p)
          if (slot[p] >= 0)
            atomicAdd(&val[slot[p]], (unsigned long long)__double2ll_rn(ldexp((double)v[p][k], F[p])));
        __syncthreads();
        for (int e = tid; e < nu; e += NT) {
          const int sl = used[e];
          const unsigned long long sum = val[sl];
          if (sum != 0ull) atomicAdd(&a.acc[(int64_t)key[sl] * d + k], sum);
          val[sl] = 0ull;
        }
        __syncthreads();
      }
    }
    for (int e = tid; e < nu; e += NT) key[used[e]] = -1;
    __syncthreads();
    if (tid == 0) n_used = 0;
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT) void backward_finish_kernel(BackwardArgs a) {
  const int d = a.d;
  const int64_t total = a.n * d;
  for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * NT) {
    const int64_t j = q / d;
    float g = a.own[q];
    const uint32_t mb = a.maxabs[j];
    if (mb != 0) {
      const int F = fixed_scale(mb, a.count[j]);
      const long long v = (long long)a.acc[q];
      g += (float)ldexp((double)v, -F);
    }
    a.grad[q] = g;
  }
}

}  // namespace

namespace {

template <int DK>
__global__ __launch_bounds__(NT) void dump_dirs_kernel(int d, int64_t first, int64_t n_cells, int R,
                                                       uint64_t seed, float *__restrict__ out) {
  for (int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x; gid < n_cells * R;
       gid += (int64_t)gridDim.x * NT) {
    const int64_t c = gid / R;
    const int ray = (int)(gid - c * R);
    float u[DK];
    mc_direction<DK>(seed, first + c, ray, d, u);
#pragma unroll
    for (int k = 0; k < DK; ++k)
      if (k < d) out[gid * d + k] = u[k];
  }
}

}  // namespace

hipError_t launch_dump_dirs(int d, int64_t first, int64_t n_cells, int R, uint64_t seed, float *out,
                            hipStream_t s) {
  const int64_t m = n_cells * R;
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<int64_t>((m + NT - 1) / NT, 1 << 20)), blk(NT);
  if (d <= 4)
    hipLaunchKernelGGL(dump_dirs_kernel<4>, grid, blk, 0, s, d, first, n_cells, R, seed, out);
  else if (d <= 8)
    hipLaunchKernelGGL(dump_dirs_kernel<8>, grid, blk, 0, s, d, first, n_cells, R, seed, out);
  else if (d <= 12)
    hipLaunchKernelGGL(dump_dirs_kernel<12>, grid, blk, 0, s, d, first, n_cells, R, seed, out);
  else
    hipLaunchKernelGGL(dump_dirs_kernel<16>, grid, blk, 0, s, d, first, n_cells, R, seed, out);
  return hipGetLastError();
}

hipError_t launch_accum(const AccumArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  int P = 1;
  while (P < a.R) P <<= 1;
  const size_t shm = (size_t)P * (sizeof(uint64_t) + sizeof(float)) + NT * sizeof(float) +
                     (NT + 1) * sizeof(int32_t);
  dim3 grid((unsigned)a.n), blk(NT);
  if (a.R <= 64) {  // one wave per cell
    const dim3 gw((unsigned)((a.n + NT / 64 - 1) / (NT / 64)));
    if (a.d <= 4)
      hipLaunchKernelGGL(accum_wave_kernel<4>, gw, blk, 0, s, a);
    else if (a.d <= 8)
      hipLaunchKernelGGL(accum_wave_kernel<8>, gw, blk, 0, s, a);
    else if (a.d <= 12)
      hipLaunchKernelGGL(accum_wave_kernel<12>, gw, blk, 0, s, a);
    else
      hipLaunchKernelGGL(accum_wave_kernel<16>, gw, blk, 0, s, a);
    return hipGetLastError();
  }
  if (a.d <= 4)
    hipLaunchKernelGGL(accum_kernel<4>, grid, blk, shm, s, a);
  else if (a.d <= 8)
    hipLaunchKernelGGL(accum_kernel<8>, grid, blk, shm, s, a);
  else if (a.d <= 12)
    hipLaunchKernelGGL(accum_kernel<12>, grid, blk, shm, s, a);
  else
    hipLaunchKernelGGL(accum_kernel<16>, grid, blk, shm, s, a);
  return hipGetLastError();
}

hipError_t launch_sample_points(const float *nodes, int64_t n, int d, int R, const float *dirs, const float *t,
                                int m, const float *tsamp, float *points, hipStream_t s) {
  const int64_t rays = n * R;
  if (rays <= 0) return hipSuccess;
  const dim3 grid((unsigned)((rays + NT - 1) / NT)), blk(NT);
  if (d <= 4)
    hipLaunchKernelGGL(sample_points_kernel<4>, grid, blk, 0, s, nodes, n, d, R, dirs, t, m, tsamp, points);
  else if (d <= 8)
    hipLaunchKernelGGL(sample_points_kernel<8>, grid, blk, 0, s, nodes, n, d, R, dirs, t, m, tsamp, points);
  else if (d <= 12)
    hipLaunchKernelGGL(sample_points_kernel<12>, grid, blk, 0, s, nodes, n, d, R, dirs, t, m, tsamp, points);
  else
    hipLaunchKernelGGL(sample_points_kernel<16>, grid, blk, 0, s, nodes, n, d, R, dirs, t, m, tsamp, points);
  return hipGetLastError();
}

hipError_t launch_backward(const BackwardArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  dim3 grid((unsigned)a.n), blk(NT);
  if (a.d <= 4)
    hipLaunchKernelGGL(backward_rays_kernel<4>, grid, blk, 0, s, a);
  else if (a.d <= 8)
    hipLaunchKernelGGL(backward_rays_kernel<8>, grid, blk, 0, s, a);
  else if (a.d <= 12)
    hipLaunchKernelGGL(backward_rays_kernel<12>, grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL(backward_rays_kernel<16>, grid, blk, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.d <= 4)
    hipLaunchKernelGGL(backward_scatter_kernel<4>, grid, blk, 0, s, a);
  else if (a.d <= 8)
    hipLaunchKernelGGL(backward_scatter_kernel<8>, grid, blk, 0, s, a);
  else if (a.d <= 12)
    hipLaunchKernelGGL(backward_scatter_kernel<12>, grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL(backward_scatter_kernel<16>, grid, blk, 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(backward_finish_kernel, dim3(1024), blk, 0, s, a);
  return hipGetLastError();
}

}  // namespace vg
