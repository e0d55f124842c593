// FP64 re-evaluation of the rays whose FP32 scan could not certify its
// argmin (near-ties, no hit, grazing winners).
//
// For each queued ray every node is evaluated in FP64 with eq. (t),
// t = (|r - x|^2 - |g - x|^2) / (2 u.(r - g)) over nodes with u.(r - g) > 0
// not in eta, the numerator in the factored form (r - g).((r - x) + (g - x))
// (no |x|^2-sized cancellation for far origins); the smallest t wins (lowest index on equality),
// then the cube clip applies, and the ray's result is overwritten.  FP
// contraction is off so that each t is the same IEEE expression as a plain
// sequential evaluation.
//
// Layout: a workgroup of 8 waves takes 8 queued rays at a time, one per wave,
// the ray's vectors held in registers; node tiles of 512 nodes (one per
// thread) are staged in LDS as [coordinate][node] and shared by the 8 rays.
// Lane l of a wave evaluates nodes l, l+64, ... of each tile and keeps a
// running top-2; the wave reduces it with cross-lane shuffles.  The batched
// variants below take one ray per wave and read their clouds directly.
// The list length is read on the device, so the launch needs no host sync: a
// fixed grid strides over the list.
#include <cstdlib>

#include "vg_internal.h"
#include "vg_philox.h"

namespace vg {
namespace {

constexpr int NT = 256;
constexpr int WAVES = NT / 64;
constexpr int TILE = 256;

struct Top2 {
  double t1, t2;
  int32_t i1;
};

__device__ __forceinline__ Top2 merge(const Top2 &a, const Top2 &b) {
  Top2 r;
  const bool take_b = (b.t1 < a.t1) || (b.t1 == a.t1 && b.i1 >= 0 && (a.i1 < 0 || b.i1 < a.i1));
  if (take_b) {
    r.t1 = b.t1;
    r.i1 = b.i1;
    r.t2 = fmin(a.t1, b.t2);
  } else {
    r.t1 = a.t1;
    r.i1 = a.i1;
    r.t2 = fmin(b.t1, a.t2);
  }
  return r;
}

// Single-problem recheck: 8 waves, one queued ray per wave; each thread
// stages one node of a 512-node tile.
constexpr int NT1 = 512;
constexpr int WAVES1 = NT1 / 64;

#pragma clang fp contract(off)
// The end of a ray's recheck (lane 0 of its wave or workgroup): the cube
// clip, the status bits and the outputs.
template <int DK>
__device__ __forceinline__ void finish_ray(const RecheckArgs &a, int64_t ray, int d, int clip, const double (&x)[DK],
                                           const double (&u)[DK], const Top2 &tp) {
  double t1 = tp.t1, t2 = tp.t2;
  int32_t i1 = tp.i1;
  if (clip) {
    double tb = __builtin_inf();
    int face = -1;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k >= d) continue;
      double tk;
      int fc;
      if (u[k] > 0.0) {
        tk = (1.0 - x[k]) / u[k];
        fc = 2 * k + 1;
      } else if (u[k] < 0.0) {
        tk = (0.0 - x[k]) / u[k];
        fc = 2 * k;
      } else {
        continue;
      }
      if (tk < tb) {
        tb = tk;
        face = fc;
      }
    }
    if (face >= 0) {
      if (tb < t1) {
        t2 = t1;
        t1 = tb;
        i1 = -2 - face;
      } else if (tb < t2) {
        t2 = tb;
      }
    }
  }
  uint8_t st = (uint8_t)((a.st_out[ray] & ~VG_ST_NO_HIT) | VG_ST_RECHECKED);
  if (i1 == -1) st |= VG_ST_NO_HIT;
  if (t2 - t1 <= 1e-9 * fabs(t1)) {
    st |= VG_ST_FP64_TIE;
    atomicAdd(a.tie_counter, 1u);
  }
  a.t_out[ray] = (float)t1;
  if (a.t64_out) a.t64_out[ray] = t1;
  a.idx_out[ray] = i1;
  a.st_out[ray] = st;
}

// Numerator and denominator of eq. (t) in FP64 for node r (coordinates v,
// as read from memory; entries k >= d unused): den = u.(r - g) and, with the
// factored numerator, num = |r - x|^2 - |g - x|^2 = (r - g).((r - x) + (g - x)).
// CELLS: the Monte-Carlo form, x = g, num = |r - g|^2.
template <int DK, bool CELLS, typename NT>
__device__ __forceinline__ void node_num_den(const NT (&v)[DK], int d, const double (&x)[DK],
                                             const double (&u)[DK], const double (&g)[DK],
                                             const double (&gx)[DK], double &num, double &den) {
  double e[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) e[k] = k < d ? (double)v[k] - g[k] : 0.0;
  den = 0.0;
#pragma unroll
  for (int k = 0; k < DK; ++k)
    if (k < d) den += u[k] * e[k];
  num = 0.0;
  if (CELLS) {
#pragma unroll
    for (int k = 0; k < DK; ++k)
      if (k < d) num += e[k] * e[k];
  } else {
#pragma unroll
    for (int k = 0; k < DK; ++k)
      if (k < d) num += e[k] * (((double)v[k] - x[k]) + gx[k]);
  }
}

// Node r with (num, den) into the running top-2 (eligible: den > 0).
__device__ __forceinline__ void top2_update(double num, double den, int32_t r, Top2 &tp) {
  if (!(den > 0.0)) return;
  // cheap filter (relaxed by 1e-12 so no candidate within rounding is lost)
  if (num > tp.t2 * (2.0 * den) * (1.0 + 1e-12) && num > 0.0) return;
  const double t = num / (2.0 * den);
  if (t < tp.t1) {
    tp.t2 = tp.t1;
    tp.t1 = t;
    tp.i1 = r;
  } else if (t < tp.t2) {
    tp.t2 = t;
  }
}

// One node against the ray, into the running top-2.
template <int DK, bool CELLS, typename NT>
__device__ __forceinline__ void eval_vals(const NT (&v)[DK], int d, int32_t r, const double (&x)[DK],
                                          const double (&u)[DK], const double (&g)[DK],
                                          const double (&gx)[DK], Top2 &tp) {
  double num, den;
  node_num_den<DK, CELLS>(v, d, x, u, g, gx, num, den);
  top2_update(num, den, r, tp);
}

// The same for a node row read in place (stride between coordinates); only
// the d coordinates of the row are read.
template <int DK, bool CELLS, typename NT>
__device__ __forceinline__ void eval_node(const NT *xr, int stride, int d, int32_t r, const double (&x)[DK],
                                          const double (&u)[DK], const double (&g)[DK],
                                          const double (&gx)[DK], Top2 &tp) {
  NT v[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) v[k] = k < d ? xr[k * stride] : NT(0);
  eval_vals<DK, CELLS>(v, d, r, x, u, g, gx, tp);
}

// The node rows a recheck reads: FP32 rows, or the exact FP64 ones.
template <typename NT>
__device__ __forceinline__ const NT *node_rows(const RecheckArgs &a);
template <>
__device__ __forceinline__ const float *node_rows<float>(const RecheckArgs &a) {
  return a.nodes;
}
template <>
__device__ __forceinline__ const double *node_rows<double>(const RecheckArgs &a) {
  return a.nodes64;
}

// DK: the dimension rounded up to 4, 8, 12 or 16 (loops guard k < d, so the
// order of every FP64 sum is the plain k = 0 .. d-1 order).  CELLS: the
// Monte-Carlo rays of a cell, x = g = x_i and eta = {i}; there the numerator
// (r - g).((r - x) + (g - x)) is exactly sum_k (r_k - g_k)^2, since
// (r_k - g_k) + 0 = r_k - g_k.
// Up to d = 8 the registers fit four waves per SIMD (two workgroups per CU),
// which hides the latency of the dependent FP64 sums; wider rays would spill.
// PART: the workgroup covers only the nodes [blockIdx.y chunk, (blockIdx.y+1)
// chunk) of the first `cap` queued rays and stores each ray's top-2 in
// parts[blockIdx.y][f] for recheck_fold_kernel (the top-2 does not depend on
// the order of the merges, so the folded result is the whole-range one).
// EXACT: d == DK, known at compile time.  The tile rows k >= d hold zeros, so
// a Monte-Carlo node's DK values are read from LDS without a branch.
template <int DK, bool CELLS, typename NT = float, bool PART = false, bool EXACT = false>
__global__ __launch_bounds__(NT1, DK <= 8 ? 4 : 1) void recheck_kernel(RecheckArgs a, int64_t chunk = 0,
                                                                      uint32_t cap = 0,
                                                                      Top2 *__restrict__ parts = nullptr) {
  __shared__ NT tile[DK * NT1];  // [k][node]: lane-contiguous reads
  // general rays: the excluded nodes of each wave's ray within the tile, one
  // bit per node (word j covers tile nodes 64 j .. 64 j + 63)
  __shared__ unsigned long long exmask[CELLS ? 1 : WAVES1][NT1 / 64];
  const NT *rows = node_rows<NT>(a);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d = EXACT ? DK : a.d;
  for (int i = d * NT1 + tid; i < DK * NT1; i += NT1) tile[i] = NT(0);
  const int64_t lo = PART ? (int64_t)blockIdx.y * chunk : 0;
  const int64_t n = PART ? (lo + chunk < a.n ? lo + chunk : a.n) : a.n;
  uint32_t cnt = a.counters[CNT_FLAGGED];
  if (PART && cnt > cap) cnt = cap;
  for (uint32_t f0 = blockIdx.x * WAVES1; f0 < cnt; f0 += gridDim.x * WAVES1) {
    const uint32_t f = f0 + w;
    const bool live = f < cnt;
    const int64_t ray = live ? a.flag_list[f] : 0;
    int n_excl = 0, clip = 0;
    int32_t gi = 0;
    // the wave's ray: origin x, direction u, generator g (x = g for CELLS)
    double x[DK], u[DK], g[DK];
    int32_t my_ex = -1;  // lane e < n_excl holds eta[e]
#pragma unroll
    for (int k = 0; k < DK; ++k) x[k] = u[k] = g[k] = 0.0;
    if (live) {
      if (CELLS) {
        gi = (int32_t)(ray / a.R);
        clip = 1;
        float uf[DK];
        cell_dir<DK>(a.dirs, a.seed, gi, a.R, (int)(ray - (int64_t)gi * a.R), d, uf);
#pragma unroll
        for (int k = 0; k < DK; ++k) u[k] = (double)uf[k];
      } else {
        gi = a.gen[ray];
        n_excl = a.n_excl;
        clip = a.clip;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          if (k < d) {
            x[k] = a.mode == RAYS_F64 ? a.o64[ray * d + k] : (double)a.o32[ray * d + k];
            u[k] = a.mode == RAYS_F64 ? a.u64[ray * d + k] : (double)a.u32[ray * d + k];
          }
        }
        if (lane < n_excl) my_ex = a.excl[ray * n_excl + lane];
      }
#pragma unroll
      for (int k = 0; k < DK; ++k) g[k] = k < d ? (double)rows[(int64_t)gi * d + k] : 0.0;
    }
    if (CELLS) {
#pragma unroll
      for (int k = 0; k < DK; ++k) x[k] = g[k];
    }
    double gx[DK];  // g - x, the same value the expression forms per node
#pragma unroll
    for (int k = 0; k < DK; ++k) gx[k] = g[k] - x[k];
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t base = lo; base < n; base += NT1) {
      const int cntn = (int)((n - base) < NT1 ? (n - base) : NT1);
      __syncthreads();
      if (tid < cntn) {
        const NT *src = rows + (base + tid) * d;
#pragma unroll
        for (int k = 0; k < DK; ++k)
          if (k < d) tile[k * NT1 + tid] = src[k];
      }
      __syncthreads();
      if (!live) continue;
      if (!CELLS) {
        // this wave's exclusion bits for the tile (LDS operations of one
        // wave complete in order)
        if (lane < NT1 / 64) exmask[w][lane] = 0ull;
        __builtin_amdgcn_wave_barrier();
        const int64_t off = (int64_t)my_ex - base;
        if (my_ex >= 0 && off >= 0 && off < cntn)
          atomicOr(&exmask[w][off >> 6], 1ull << (off & 63));
        __builtin_amdgcn_wave_barrier();
      }
      // two nodes per step, q and q + 64: their FP64 sums are independent
      // chains that overlap; the top-2 still takes the nodes in index order
      for (int q = lane; q < cntn; q += 128) {
        const bool has2 = q + 64 < cntn;
        const int q2 = has2 ? q + 64 : q;
        const int32_t r = (int32_t)(base + q), r2 = (int32_t)(base + q2);
        bool skip, skip2;
        if (CELLS) {
          skip = r == gi;
          skip2 = r2 == gi;
        } else {
          const int j = (q - lane) >> 6;  // wave-uniform word index
          skip = (exmask[w][j] >> lane) & 1ull;
          skip2 = j + 1 < NT1 / 64 ? ((exmask[w][j + 1] >> lane) & 1ull) : false;
        }
        skip2 |= !has2;
        // CELLS: all DK rows, no branch (the rows k >= d of the tile are zero);
        // general rays read only the d rows (their register budget is spent)
        NT v[DK], w[DK];
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          v[k] = (CELLS || EXACT || k < d) ? tile[k * NT1 + q] : NT(0);
          w[k] = (CELLS || EXACT || k < d) ? tile[k * NT1 + q2] : NT(0);
        }
        double num, den, num2, den2;
        node_num_den<DK, CELLS>(v, d, x, u, g, gx, num, den);
        node_num_den<DK, CELLS>(w, d, x, u, g, gx, num2, den2);
        if (!skip) top2_update(num, den, r, tp);
        if (!skip2) top2_update(num2, den2, r2, tp);
      }
    }
    if (live) {
      for (int off = 32; off > 0; off >>= 1) {
        Top2 o;
        o.t1 = __shfl_xor(tp.t1, off);
        o.t2 = __shfl_xor(tp.t2, off);
        o.i1 = __shfl_xor(tp.i1, off);
        tp = merge(tp, o);
      }
      if (lane == 0) {
        if (PART)
          parts[(int64_t)blockIdx.y * cap + f] = tp;
        else
          finish_ray<DK>(a, ray, d, clip, x, u, tp);
      }
    }
  }
}

// Large clouds: one queued ray per workgroup, its 512 threads striding over
// the nodes read from memory (a few queued rays then still fill the GPU),
// merged by shuffles and across waves in LDS.  The same node expression and
// finish as recheck_kernel, and the top-2 does not depend on the order of
// the merges, so the results are the same.  NT = double reads the exact
// FP64 rows (general rays whose FP32 rows were rounded).
template <int DK, bool CELLS, typename NT = float>
__global__ __launch_bounds__(NT1) void recheck_wide_kernel(RecheckArgs a, uint32_t f_begin = 0) {
  const NT *rows = node_rows<NT>(a);
  __shared__ double st1[WAVES1], st2[WAVES1];
  __shared__ int32_t si1[WAVES1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d = a.d;
  const int64_t n = a.n;
  const uint32_t cnt = a.counters[CNT_FLAGGED];
  for (uint32_t f = f_begin + blockIdx.x; f < cnt; f += gridDim.x) {
    const int64_t ray = a.flag_list[f];
    int n_excl = 0, clip = 0;
    int32_t gi;
    double x[DK], u[DK], g[DK];
    int32_t ex[VG_MAX_DIM];
#pragma unroll
    for (int e = 0; e < VG_MAX_DIM; ++e) ex[e] = -1;
    if (CELLS) {
      gi = (int32_t)(ray / a.R);
      clip = 1;
      float uf[DK];
      cell_dir<DK>(a.dirs, a.seed, gi, a.R, (int)(ray - (int64_t)gi * a.R), d, uf);
#pragma unroll
      for (int k = 0; k < DK; ++k) u[k] = (double)uf[k];
    } else {
      gi = a.gen[ray];
      n_excl = a.n_excl;
      clip = a.clip;
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        x[k] = k < d ? (a.mode == RAYS_F64 ? a.o64[ray * d + k] : (double)a.o32[ray * d + k]) : 0.0;
        u[k] = k < d ? (a.mode == RAYS_F64 ? a.u64[ray * d + k] : (double)a.u32[ray * d + k]) : 0.0;
      }
#pragma unroll
      for (int e = 0; e < VG_MAX_DIM; ++e)
        if (e < n_excl) ex[e] = a.excl[ray * n_excl + e];
    }
#pragma unroll
    for (int k = 0; k < DK; ++k) g[k] = k < d ? (double)rows[(int64_t)gi * d + k] : 0.0;
    if (CELLS) {
#pragma unroll
      for (int k = 0; k < DK; ++k) x[k] = g[k];
    }
    double gx[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) gx[k] = g[k] - x[k];
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t r = tid; r < n; r += NT1) {
      bool skip;
      if (CELLS) {
        skip = r == gi;
      } else {
        skip = false;
#pragma unroll
        for (int e = 0; e < VG_MAX_DIM; ++e) skip |= (e < n_excl && ex[e] == r);
      }
      if (!skip) eval_node<DK, CELLS>(rows + r * d, 1, d, (int32_t)r, x, u, g, gx, tp);
    }
    for (int off = 32; off > 0; off >>= 1) {
      Top2 o;
      o.t1 = __shfl_xor(tp.t1, off);
      o.t2 = __shfl_xor(tp.t2, off);
      o.i1 = __shfl_xor(tp.i1, off);
      tp = merge(tp, o);
    }
    __syncthreads();  // the previous ray's merge has read the LDS slots
    if (lane == 0) {
      st1[w] = tp.t1;
      st2[w] = tp.t2;
      si1[w] = tp.i1;
    }
    __syncthreads();
    if (tid == 0) {
      Top2 all{st1[0], st2[0], si1[0]};
      for (int q = 1; q < WAVES1; ++q) all = merge(all, Top2{st1[q], st2[q], si1[q]});
      finish_ray<DK>(a, ray, d, clip, x, u, all);
    }
  }
}

#pragma clang fp contract(off)
// Batched Monte-Carlo rays: a queue entry is (problem << 40 | ray); each wave
// takes one entry and reads that cloud's nodes directly (entries of one
// workgroup may belong to different clouds, so no LDS tile is shared).
__global__ __launch_bounds__(NT) void recheck_batched_kernel(const BatchProblem *probs,
                                                             const uint32_t *counters,
                                                             const int64_t *flag_list,
                                                             uint32_t *tie_counter) {
  const int lane = threadIdx.x & 63;
  const uint32_t cnt = counters[CNT_FLAGGED];
  const uint32_t nw = gridDim.x * WAVES;
  for (uint32_t f = blockIdx.x * WAVES + (threadIdx.x >> 6); f < cnt; f += nw) {
    const int64_t code = flag_list[f];
    const int p = (int)(code >> 40);
    const int64_t ray = code & ((int64_t(1) << 40) - 1);
    const CellScanArgs &a = probs[p].a;
    const int d = a.d;
    const int64_t cell = ray / a.R;
    double x[VG_MAX_DIM], u[VG_MAX_DIM];
    float uf[VG_MAX_DIM];
    cell_dir<VG_MAX_DIM>(a.dirs, a.seed, cell, a.R, (int)(ray - cell * a.R), d, uf);
    for (int k = 0; k < d; ++k) {
      x[k] = (double)a.nodes[cell * d + k];
      u[k] = (double)uf[k];
    }
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t r = lane; r < a.n; r += 64) {
      if (r == cell) continue;
      const float *xr = a.nodes + r * d;
      double den = 0.0;
      for (int k = 0; k < d; ++k) den += u[k] * ((double)xr[k] - x[k]);
      if (!(den > 0.0)) continue;
      double num = 0.0;  // (r - g).((r - x) + (g - x)) with x = g
      for (int k = 0; k < d; ++k)
        num += ((double)xr[k] - x[k]) * (((double)xr[k] - x[k]) + (x[k] - x[k]));
      if (num > tp.t2 * (2.0 * den) * (1.0 + 1e-12) && num > 0.0) continue;
      const double t = num / (2.0 * den);
      if (t < tp.t1) {
        tp.t2 = tp.t1;
        tp.t1 = t;
        tp.i1 = (int32_t)r;
      } else if (t < tp.t2) {
        tp.t2 = t;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      Top2 o;
      o.t1 = __shfl_xor(tp.t1, off);
      o.t2 = __shfl_xor(tp.t2, off);
      o.i1 = __shfl_xor(tp.i1, off);
      tp = merge(tp, o);
    }
    if (lane == 0) {
      double t1 = tp.t1, t2 = tp.t2;
      int32_t i1 = tp.i1;
      double tb = __builtin_inf();
      int face = -1;
      for (int k = 0; k < d; ++k) {
        double tk;
        int fc;
        if (u[k] > 0.0) {
          tk = (1.0 - x[k]) / u[k];
          fc = 2 * k + 1;
        } else if (u[k] < 0.0) {
          tk = (0.0 - x[k]) / u[k];
          fc = 2 * k;
        } else {
          continue;
        }
        if (tk < tb) {
          tb = tk;
          face = fc;
        }
      }
      if (face >= 0) {
        if (tb < t1) {
          t2 = t1;
          t1 = tb;
          i1 = -2 - face;
        } else if (tb < t2) {
          t2 = tb;
        }
      }
      uint8_t st = (uint8_t)((a.st_out[ray] & ~VG_ST_NO_HIT) | VG_ST_RECHECKED);
      if (i1 == -1) st |= VG_ST_NO_HIT;
      if (t2 - t1 <= 1e-9 * fabs(t1)) {
        st |= VG_ST_FP64_TIE;
        atomicAdd(tie_counter, 1u);
      }
      a.t_out[ray] = (float)t1;
      a.idx_out[ray] = i1;
      a.st_out[ray] = st;
    }
  }
}


// Batched general rays: a queue entry is (problem << 40 | ray); each wave
// takes one entry and evaluates every node of that problem in FP64 with the
// same expressions, filter and clip rule as recheck_kernel (loops unrolled
// over VG_MAX_DIM with a k < d guard, so the order of the sums is the same).
__global__ __launch_bounds__(NT) void recheck_rays_batched_kernel(const RayBatchProblem *probs,
                                                                  const uint32_t *counters,
                                                                  const int64_t *flag_list,
                                                                  uint32_t *tie_counter) {
  const int lane = threadIdx.x & 63;
  const uint32_t cnt = counters[CNT_FLAGGED];
  const uint32_t nw = gridDim.x * WAVES;
  for (uint32_t f = blockIdx.x * WAVES + (threadIdx.x >> 6); f < cnt; f += nw) {
    const int64_t code = flag_list[f];
    const int p = (int)(code >> 40);
    const int64_t ray = code & ((int64_t(1) << 40) - 1);
    const RayScanArgs &a = probs[p].a;
    const int d = a.d;
    const int n_excl = a.n_excl;
    const int32_t gi = a.gen[ray];  // in range: rays with a bad generator are never queued
    double x[VG_MAX_DIM], u[VG_MAX_DIM], g[VG_MAX_DIM];
    int32_t ex[VG_MAX_DIM];
#pragma unroll
    for (int k = 0; k < VG_MAX_DIM; ++k) {
      x[k] = k < d ? (double)a.o32[ray * d + k] : 0.0;
      u[k] = k < d ? (double)a.u32[ray * d + k] : 0.0;
      g[k] = k < d ? (double)a.nodes[(int64_t)gi * d + k] : 0.0;
      ex[k] = k < n_excl ? a.excl[ray * n_excl + k] : -1;
    }
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t r = lane; r < a.n; r += 64) {
      bool skip = false;
#pragma unroll
      for (int e = 0; e < VG_MAX_DIM; ++e) skip |= (e < n_excl && ex[e] == r);
      if (skip) continue;
      const float *xr = a.nodes + r * d;
      double den = 0.0;
#pragma unroll
      for (int k = 0; k < VG_MAX_DIM; ++k)
        if (k < d) den += u[k] * ((double)xr[k] - g[k]);
      if (!(den > 0.0)) continue;
      double num = 0.0;
#pragma unroll
      for (int k = 0; k < VG_MAX_DIM; ++k)
        if (k < d) num += ((double)xr[k] - g[k]) * (((double)xr[k] - x[k]) + (g[k] - x[k]));
      if (num > tp.t2 * (2.0 * den) * (1.0 + 1e-12) && num > 0.0) continue;
      const double t = num / (2.0 * den);
      if (t < tp.t1) {
        tp.t2 = tp.t1;
        tp.t1 = t;
        tp.i1 = (int32_t)r;
      } else if (t < tp.t2) {
        tp.t2 = t;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      Top2 o;
      o.t1 = __shfl_xor(tp.t1, off);
      o.t2 = __shfl_xor(tp.t2, off);
      o.i1 = __shfl_xor(tp.i1, off);
      tp = merge(tp, o);
    }
    if (lane == 0) {
      double t1 = tp.t1, t2 = tp.t2;
      int32_t i1 = tp.i1;
      if (a.clip) {
        double tb = __builtin_inf();
        int face = -1;
        for (int k = 0; k < d; ++k) {
          double tk;
          int fc;
          if (u[k] > 0.0) {
            tk = (1.0 - x[k]) / u[k];
            fc = 2 * k + 1;
          } else if (u[k] < 0.0) {
            tk = (0.0 - x[k]) / u[k];
            fc = 2 * k;
          } else {
            continue;
          }
          if (tk < tb) {
            tb = tk;
            face = fc;
          }
        }
        if (face >= 0) {
          if (tb < t1) {
            t2 = t1;
            t1 = tb;
            i1 = -2 - face;
          } else if (tb < t2) {
            t2 = tb;
          }
        }
      }
      uint8_t st = (uint8_t)((a.st_out[ray] & ~VG_ST_NO_HIT) | VG_ST_RECHECKED);
      if (i1 == -1) st |= VG_ST_NO_HIT;
      if (t2 - t1 <= 1e-9 * fabs(t1)) {
        st |= VG_ST_FP64_TIE;
        atomicAdd(tie_counter, 1u);
      }
      a.t_out[ray] = (float)t1;
      a.idx_out[ray] = i1;
      a.st_out[ray] = st;
    }
  }
}

// Monte-Carlo rays over fewer than 2^18 nodes, targeted: a queued ray first
// runs an FP32 pass over all nodes that keeps only the candidates that can
// still be its winner, and only those are evaluated in FP64 (normally one to
// three instead of every node).
//
// FP32 pass: with e = r - x_i the value s = (u.e)/|e|^2 = 1/(2 t) is
// computed with FMAs, and |s~ - s| <= delta = c / |e|, c = (2d + 8) 2^-24
// (to first order: u.e within (d + 1) 2^-24 |e|, |e|^2 within (d + 2)
// 2^-24 relative, the reciprocal square root, its square and the product a
// few ulps; |u| = 1).  L is the largest lower bound s~ - 2 delta seen
// (initially the cube's exit, lowered by 2^-18 for its rounding), and a
// node is kept while s~ + 4 delta >= L: the winner is always kept (its s
// is at least every lower bound), and a dropped node has
// s <= s~ + delta < L - 3 delta <= s(winner) - 3 delta, so it is worse than
// the winner by far more than FP64 rounding and cannot be the FP64 argmin,
// tie with it, or sit within the FP64 tie gap 1e-9 of it.  The kept nodes
// are evaluated with the same FP64 expression as the full recheck, merged
// with the same lowest-index rule and finished by the same finish_ray, so
// the result is the full recheck's.  A lane that would keep more than KC
// nodes at once marks its ray, which then gets the full FP64 pass.
constexpr int KC = 4;

template <int D>
__global__ __launch_bounds__(NT1) void band_cells_kernel(RecheckArgs a) {
  __shared__ float tile[D * NT1];  // [k][node]
  __shared__ int any_over;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n = a.n;
  const uint32_t cnt = a.counters[CNT_FLAGGED];
  constexpr float c_b = (2.f * D + 8.f) * 0x1p-24f;
  for (uint32_t f0 = blockIdx.x * WAVES1; f0 < cnt; f0 += gridDim.x * WAVES1) {
    const uint32_t f = f0 + w;
    const bool live = f < cnt;
    const int64_t ray = live ? a.flag_list[f] : 0;
    const int32_t gi = (int32_t)(ray / a.R);
    float uf[D], xf[D];
    if (live) {
      cell_dir<D>(a.dirs, a.seed, gi, a.R, (int)(ray - (int64_t)gi * a.R), D, uf);
#pragma unroll
      for (int k = 0; k < D; ++k) xf[k] = a.nodes[(int64_t)gi * D + k];
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) uf[k] = xf[k] = 0.f;
    }
    // the cube's exit in the s domain, lowered by a margin for its rounding
    float L = 0.f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (uf[k] != 0.f) {
        const float h = uf[k] > 0.f ? 1.f - xf[k] : xf[k];
        L = fmaxf(L, fabsf(uf[k]) / (2.f * h));
      }
    }
    L *= 1.f - 0x1p-18f;
    float cs[KC];
    int32_t ci[KC];
    int nc = 0;
    bool over = false;
    if (tid == 0) any_over = 0;
    for (int64_t base = 0; base < n; base += NT1) {
      const int cntn = (int)((n - base) < NT1 ? (n - base) : NT1);
      __syncthreads();
      if (tid < cntn) {
        const float *src = a.nodes + (base + tid) * D;
#pragma unroll
        for (int k = 0; k < D; ++k) tile[k * NT1 + tid] = src[k];
      }
      __syncthreads();
      if (!live) continue;
      for (int q = lane; q < cntn; q += 64) {
        const int32_t r = (int32_t)(base + q);
        float n2 = 0.f, den = 0.f;
        bool same = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const float e = tile[k * NT1 + q] - xf[k];
          same &= e == 0.f;
          n2 = __builtin_fmaf(e, e, n2);
          den = __builtin_fmaf(uf[k], e, den);
        }
        // x_i itself and its exact duplicates are never eligible (u.e = 0);
        // a node so close that |e|^2 underflows gets the full FP64 pass
        if (r == gi || same) continue;
        if (!(n2 >= 0x1p-100f)) {
          over = true;
          continue;
        }
        const float rs = __builtin_amdgcn_rsqf(n2);
        const float sv = den * (rs * rs);
        const float delta = c_b * rs;
        const float lo = sv - 2.f * delta;  // below s by at least delta
        if (lo > L) {
          L = lo;
          int m = 0;
#pragma unroll
          for (int e = 0; e < KC; ++e) {
            const bool keep = e < nc && cs[e] >= L;
            if (keep) {
              cs[m] = cs[e];
              ci[m] = ci[e];
            }
            m += keep ? 1 : 0;
          }
          nc = m;
        }
        const float hi = sv + 4.f * delta;
        if (hi >= L) {
          if (nc < KC) {
#pragma unroll
            for (int e = 0; e < KC; ++e)
              if (e == nc) {
                cs[e] = hi;
                ci[e] = r;
              }
            ++nc;
          } else {
            over = true;
          }
        }
      }
    }
    if (!live) continue;
    // the wave's bound, then the kept nodes in FP64
    float Lw = L;
    for (int off = 32; off > 0; off >>= 1) Lw = fmaxf(Lw, __shfl_xor(Lw, off));
    const bool wave_over = __ballot(over) != 0ull;
    double x[D], u[D], g[D], gx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      u[k] = (double)uf[k];
      g[k] = x[k] = (double)xf[k];
      gx[k] = 0.0;
    }
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    if (!wave_over) {
#pragma unroll
      for (int e = 0; e < KC; ++e)
        if (e < nc && cs[e] >= Lw) eval_node<D, true>(a.nodes + (int64_t)ci[e] * D, 1, D, ci[e], x, u, g, gx, tp);
    } else {
      for (int64_t r = lane; r < n; r += 64)
        if (r != gi) eval_node<D, true>(a.nodes + r * D, 1, D, (int32_t)r, x, u, g, gx, tp);
    }
    for (int off = 32; off > 0; off >>= 1) {
      Top2 o;
      o.t1 = __shfl_xor(tp.t1, off);
      o.t2 = __shfl_xor(tp.t2, off);
      o.i1 = __shfl_xor(tp.i1, off);
      tp = merge(tp, o);
    }
    if (lane == 0) finish_ray<D>(a, ray, D, 1, x, u, tp);
  }
}

// Few queued general rays over many nodes (the caller knows the queue length
// cnt): workgroup (x, y) takes queued rays x, x + gridDim.x, ... over the
// nodes [y chunk, (y+1) chunk), with the wide kernel's striding and merges,
// and stores the part's top-2 in parts[y][f]; recheck_fold_kernel merges the
// parts of each ray (the top-2 does not depend on the order of the merges,
// so the results are the wide kernel's) and finishes it.
// EXACT: d == DK, known at compile time (no guarded coordinate reads).
template <int DK, typename NT = float, bool EXACT = false>
__global__ __launch_bounds__(NT1) void recheck_part_kernel(RecheckArgs a, int64_t chunk, uint32_t cnt,
                                                           Top2 *__restrict__ parts) {
  __shared__ double st1[WAVES1], st2[WAVES1];
  __shared__ int32_t si1[WAVES1];
  const NT *rows = node_rows<NT>(a);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d = EXACT ? DK : a.d;
  const int64_t lo = (int64_t)blockIdx.y * chunk;
  const int64_t hi = lo + chunk < a.n ? lo + chunk : a.n;
  for (uint32_t f = blockIdx.x; f < cnt; f += gridDim.x) {
    const int64_t ray = a.flag_list[f];
    const int32_t gi = a.gen[ray];
    const int n_excl = a.n_excl;
    double x[DK], u[DK], g[DK];
    int32_t ex[VG_MAX_DIM];
#pragma unroll
    for (int e = 0; e < VG_MAX_DIM; ++e) ex[e] = e < n_excl ? a.excl[ray * n_excl + e] : -1;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      x[k] = k < d ? (a.mode == RAYS_F64 ? a.o64[ray * d + k] : (double)a.o32[ray * d + k]) : 0.0;
      u[k] = k < d ? (a.mode == RAYS_F64 ? a.u64[ray * d + k] : (double)a.u32[ray * d + k]) : 0.0;
      g[k] = k < d ? (double)rows[(int64_t)gi * d + k] : 0.0;
    }
    double gx[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) gx[k] = g[k] - x[k];
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t r = lo + tid; r < hi; r += NT1) {
      bool skip = false;
#pragma unroll
      for (int e = 0; e < VG_MAX_DIM; ++e) skip |= (e < n_excl && ex[e] == r);
      if (!skip) eval_node<DK, false>(rows + r * d, 1, d, (int32_t)r, x, u, g, gx, tp);
    }
    for (int off = 32; off > 0; off >>= 1) {
      Top2 o;
      o.t1 = __shfl_xor(tp.t1, off);
      o.t2 = __shfl_xor(tp.t2, off);
      o.i1 = __shfl_xor(tp.i1, off);
      tp = merge(tp, o);
    }
    __syncthreads();  // the previous ray's merge has read the LDS slots
    if (lane == 0) {
      st1[w] = tp.t1;
      st2[w] = tp.t2;
      si1[w] = tp.i1;
    }
    __syncthreads();
    if (tid == 0) {
      Top2 all{st1[0], st2[0], si1[0]};
      for (int q = 1; q < WAVES1; ++q) all = merge(all, Top2{st1[q], st2[q], si1[q]});
      parts[(int64_t)blockIdx.y * cnt + f] = all;
    }
  }
}

// The parts are stored as parts[p][f], f < stride.  CELLS: the Monte-Carlo
// rays, whose queue length is read on the device (the first `stride` of it).
template <int DK, bool CELLS = false>
__global__ __launch_bounds__(256) void recheck_fold_kernel(RecheckArgs a, int P, uint32_t stride,
                                                           const Top2 *__restrict__ parts) {
  const uint32_t f = blockIdx.x * 256u + threadIdx.x;
  uint32_t cnt = stride;
  if (CELLS && a.counters[CNT_FLAGGED] < cnt) cnt = a.counters[CNT_FLAGGED];
  if (f >= cnt) return;
  const int64_t ray = a.flag_list[f];
  const int d = a.d;
  double x[DK], u[DK];
  if (CELLS) {
    const int64_t gi = ray / a.R;
    float uf[DK];
    cell_dir<DK>(a.dirs, a.seed, gi, a.R, (int)(ray - gi * a.R), d, uf);
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      x[k] = k < d ? (double)a.nodes[gi * d + k] : 0.0;
      u[k] = (double)uf[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      x[k] = k < d ? (a.mode == RAYS_F64 ? a.o64[ray * d + k] : (double)a.o32[ray * d + k]) : 0.0;
      u[k] = k < d ? (a.mode == RAYS_F64 ? a.u64[ray * d + k] : (double)a.u32[ray * d + k]) : 0.0;
    }
  }
  Top2 tp = parts[f];
  for (int p = 1; p < P; ++p) tp = merge(tp, parts[(int64_t)p * stride + f]);
  finish_ray<DK>(a, ray, d, CELLS ? 1 : a.clip, x, u, tp);
}

// Monte-Carlo rays over many nodes, split with no host sync: the first
// kCellsSplitCap queued rays go to the PART form of recheck_kernel (8 rays
// per workgroup sharing each LDS node tile, over P node chunks) and the fold;
// the rest of a longer queue to the wide kernel.
constexpr uint32_t kCellsSplitCap = 8192;
constexpr int64_t kCellsSplitChunk = 16384;
int cells_split_parts(int64_t n) {
  if (n < (int64_t(1) << 18)) return 1;
  int64_t P = n / kCellsSplitChunk;
  return P > 64 ? 64 : (int)P;
}

// Parts of the split recheck of cnt queued general rays over n nodes (1: no
// split): only where one workgroup per ray would stream many nodes, and
// P cnt <= kSplitRecheckEntries.
constexpr int64_t kSplitRecheckEntries = int64_t(1) << 20;
int split_recheck_parts(uint32_t cnt, int64_t n) {
  if (cnt == 0 || n < (int64_t(1) << 18)) return 1;
  int64_t P = 8192 / cnt;
  if (P > 64) P = 64;
  if (P > n / 4096) P = n / 4096;
  if (P > kSplitRecheckEntries / cnt) P = kSplitRecheckEntries / cnt;
  return P > 1 ? (int)P : 1;
}

}  // namespace

hipError_t launch_recheck_batched(const BatchProblem *probs_dev, const uint32_t *counters,
                                  const int64_t *flag_list, uint32_t *tie_counter, int grid,
                                  hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(recheck_batched_kernel, dim3(grid), dim3(NT), 0, s, probs_dev, counters,
                     flag_list, tie_counter);
  return hipGetLastError();
}

size_t recheck_split_reserve(int64_t m, int64_t n) {
  if (n < (int64_t(1) << 18)) return 0;
  const int64_t e = m * 64 < kSplitRecheckEntries ? m * 64 : kSplitRecheckEntries;
  return (size_t)e * sizeof(Top2);
}

bool launch_recheck_split(const RecheckArgs &a, uint32_t cnt, void *parts, size_t parts_bytes, hipStream_t s,
                          hipError_t &err) {
  err = hipSuccess;
  const int P = split_recheck_parts(cnt, a.n);
  if (P <= 1 || a.mode == RAYS_CELLS || (a.nodes64 && a.d > 8) || !parts ||
      parts_bytes < (size_t)P * cnt * sizeof(Top2))
    return false;
  const int64_t chunk = ((a.n + P - 1) / P + NT1 - 1) / NT1 * NT1;
  const int parts_n = (int)((a.n + chunk - 1) / chunk);
  const unsigned gx = cnt < 8192u / (unsigned)parts_n ? cnt : 8192u / (unsigned)parts_n;
  const dim3 grid(gx, (unsigned)parts_n), blk(NT1), gfold((cnt + 255) / 256), bfold(256);
  Top2 *pt = static_cast<Top2 *>(parts);
#define VG_SPLIT_RECHECK(DKV, NTV, EX, DW)                                                           \
  do {                                                                                              \
    hipLaunchKernelGGL((recheck_part_kernel<DKV, NTV, EX>), grid, blk, 0, s, a, chunk, cnt, pt);     \
    hipLaunchKernelGGL(recheck_fold_kernel<DW>, gfold, bfold, 0, s, a, parts_n, cnt, (const Top2 *)pt); \
  } while (0)
#define VG_SPLIT_RECHECK_EXACT(NTV)                                                                 \
  do {                                                                                              \
    switch (a.d) {                                                                                  \
      case 2: VG_SPLIT_RECHECK(2, NTV, true, 4); break;                                             \
      case 3: VG_SPLIT_RECHECK(3, NTV, true, 4); break;                                             \
      case 4: VG_SPLIT_RECHECK(4, NTV, true, 4); break;                                             \
      case 5: VG_SPLIT_RECHECK(5, NTV, true, 8); break;                                             \
      case 6: VG_SPLIT_RECHECK(6, NTV, true, 8); break;                                             \
      case 7: VG_SPLIT_RECHECK(7, NTV, true, 8); break;                                             \
      default: VG_SPLIT_RECHECK(8, NTV, true, 8); break;                                            \
    }                                                                                               \
  } while (0)
  if (a.nodes64) {
    VG_SPLIT_RECHECK_EXACT(double);  // d <= 8 here
  } else if (a.d <= 8) {
    VG_SPLIT_RECHECK_EXACT(float);
  } else if (a.d <= 12) {
    VG_SPLIT_RECHECK(12, float, false, 12);
  } else {
    VG_SPLIT_RECHECK(16, float, false, 16);
  }
#undef VG_SPLIT_RECHECK_EXACT
#undef VG_SPLIT_RECHECK
  err = hipGetLastError();
  return true;
}

size_t recheck_cells_reserve(int64_t m, int64_t n) {
  const int P = cells_split_parts(n);
  if (P <= 1) return 0;
  const int64_t cap = m < kCellsSplitCap ? m : kCellsSplitCap;
  return (size_t)P * cap * sizeof(Top2);
}

bool launch_recheck_cells_split(const RecheckArgs &a, int64_t m, void *parts, size_t parts_bytes, hipStream_t s,
                                hipError_t &err) {
  err = hipSuccess;
  const int P = cells_split_parts(a.n);
  const uint32_t cap = (uint32_t)(m < kCellsSplitCap ? m : kCellsSplitCap);
  if (a.mode != RAYS_CELLS || P <= 1 || !parts || parts_bytes < (size_t)P * cap * sizeof(Top2)) return false;
  const int64_t chunk = ((a.n + P - 1) / P + NT1 - 1) / NT1 * NT1;
  const int parts_n = (int)((a.n + chunk - 1) / chunk);
  const unsigned groups = (cap + WAVES1 - 1) / WAVES1;
  const dim3 grid(groups < 256u ? groups : 256u, (unsigned)parts_n), blk(NT1), gfold((cap + 255) / 256), bfold(256);
  const int64_t rest = m - (int64_t)cap;
  const dim3 gridw((unsigned)(rest < 4096 ? rest : 4096));
  Top2 *pt = static_cast<Top2 *>(parts);
#define VG_CELLS_SPLIT(DKV, EX, DW)                                                                         \
  do {                                                                                                      \
    hipLaunchKernelGGL((recheck_kernel<DKV, true, float, true, EX>), grid, blk, 0, s, a, chunk, cap, pt);    \
    hipLaunchKernelGGL((recheck_fold_kernel<DW, true>), gfold, bfold, 0, s, a, parts_n, cap, (const Top2 *)pt); \
    if (rest > 0) hipLaunchKernelGGL((recheck_wide_kernel<DW, true>), gridw, blk, 0, s, a, cap);              \
  } while (0)
  switch (a.d) {
    case 2: VG_CELLS_SPLIT(2, true, 4); break;
    case 3: VG_CELLS_SPLIT(3, true, 4); break;
    case 4: VG_CELLS_SPLIT(4, true, 4); break;
    case 5: VG_CELLS_SPLIT(5, true, 8); break;
    case 6: VG_CELLS_SPLIT(6, true, 8); break;
    case 7: VG_CELLS_SPLIT(7, true, 8); break;
    case 8: VG_CELLS_SPLIT(8, true, 8); break;
    default:
      if (a.d <= 12)
        VG_CELLS_SPLIT(12, false, 12);
      else
        VG_CELLS_SPLIT(16, false, 16);
  }
#undef VG_CELLS_SPLIT
  err = hipGetLastError();
  return true;
}

hipError_t launch_recheck(const RecheckArgs &a, int max_grid, hipStream_t s, int64_t queued) {
  if (max_grid <= 0) return hipSuccess;
  const dim3 grid((max_grid + WAVES1 - 1) / WAVES1), blk(NT1);
  const bool cells = a.mode == RAYS_CELLS;
  // large clouds: a workgroup per queued ray when the queue is short (or of
  // unknown length); a queue of 2048 rays or more fills the GPU with 8 rays
  // per workgroup, each node tile then read once for 8 rays
  const bool wide = a.n >= (int64_t(1) << 18) && (queued < 0 || queued < 2048);
  const dim3 gridw(max_grid);
  // general rays, d <= 8, 8 rays per LDS tile: d a compile-time constant
#define VG_RECHECK_EXACT(NTV)                                                                  \
  do {                                                                                        \
    switch (a.d) {                                                                            \
      case 2: hipLaunchKernelGGL((recheck_kernel<2, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      case 3: hipLaunchKernelGGL((recheck_kernel<3, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      case 4: hipLaunchKernelGGL((recheck_kernel<4, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      case 5: hipLaunchKernelGGL((recheck_kernel<5, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      case 6: hipLaunchKernelGGL((recheck_kernel<6, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      case 7: hipLaunchKernelGGL((recheck_kernel<7, false, NTV, false, true>), grid, blk, 0, s, a); break; \
      default: hipLaunchKernelGGL((recheck_kernel<8, false, NTV, false, true>), grid, blk, 0, s, a); break; \
    }                                                                                         \
  } while (0)
  if (a.nodes64) {  // exact FP64 rows: general rays, d <= 8
    if (cells || a.d > 8) return hipErrorInvalidValue;
    VG_RECHECK_EXACT(double);
    return hipGetLastError();
  }
  if (!cells && !wide && a.d <= 8) {
    VG_RECHECK_EXACT(float);
    return hipGetLastError();
  }
#undef VG_RECHECK_EXACT
  // Monte-Carlo rays over fewer than 2^18 nodes: the targeted band recheck
  // (VG_FULL_RECHECK set: every node in FP64, for comparison)
  if (cells && !wide && std::getenv("VG_FULL_RECHECK") == nullptr) {
    switch (a.d) {
#define VG_BAND(DV) \
  case DV: hipLaunchKernelGGL(band_cells_kernel<DV>, grid, blk, 0, s, a); break;
      VG_BAND(2) VG_BAND(3) VG_BAND(4) VG_BAND(5) VG_BAND(6) VG_BAND(7) VG_BAND(8) VG_BAND(9)
      VG_BAND(10) VG_BAND(11) VG_BAND(12) VG_BAND(13) VG_BAND(14) VG_BAND(15) VG_BAND(16)
#undef VG_BAND
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
#define VG_RECHECK(DKV)                                                            \
  do {                                                                            \
    if (wide && cells)                                                            \
      hipLaunchKernelGGL((recheck_wide_kernel<DKV, true>), gridw, blk, 0, s, a);  \
    else if (wide)                                                                \
      hipLaunchKernelGGL((recheck_wide_kernel<DKV, false>), gridw, blk, 0, s, a); \
    else if (cells)                                                               \
      hipLaunchKernelGGL((recheck_kernel<DKV, true>), grid, blk, 0, s, a);        \
    else                                                                          \
      hipLaunchKernelGGL((recheck_kernel<DKV, false>), grid, blk, 0, s, a);       \
  } while (0)
  if (a.d <= 4)
    VG_RECHECK(4);
  else if (a.d <= 8)
    VG_RECHECK(8);
  else if (a.d <= 12)
    VG_RECHECK(12);
  else
    VG_RECHECK(16);
#undef VG_RECHECK
  return hipGetLastError();
}

hipError_t launch_recheck_rays_batched(const RayBatchProblem *probs_dev, const uint32_t *counters,
                                       const int64_t *flag_list, uint32_t *tie_counter, int grid,
                                       hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(recheck_rays_batched_kernel, dim3(grid), dim3(NT), 0, s, probs_dev, counters,
                     flag_list, tie_counter);
  return hipGetLastError();
}

}  // namespace vg
