// RayCast of arbitrary rays in FP32 on the vector ALUs (gfx950).
//
// Each ray has its own origin x (a Voronoi vertex during the exhaustive
// search), so the contraction X.R^T has no reuse across rays; the scan
// evaluates eq. (t) directly, with the numerator as a difference of squares
// in factored form,
//     num = |r - x|^2 - |g - x|^2 = sum_k (r_k - g_k) ((r_k - x_k) + (g_k - x_k)),
//     den = sum_k u_k (r_k - g_k),
// which stays accurate when the origin is far from the nodes (hull vertices
// of the unbounded diagram reach |x| ~ 1e6): no |x|^2-sized terms cancel.
// Eligible nodes have den > 0 and are not in eta (sorted, walked alongside
// the ascending node index).  One thread per ray; nodes stream through LDS in
// tiles of 256 and are broadcast to the 64 lanes of a wave.
//
// The running top-2 avoids a division per pair: a node can only enter the
// top-2 if num < t2 * den (den > 0); only then is t = num/den formed.
// A ray is queued for the FP64 recheck when
//   * its two best candidates are within their FP32 error bounds (or a
//     relative gap tau),
//   * the winner's own FP32 error bound exceeds tau t (far origins),
//   * some nearly grazing node (|den| within its rounding bound, so its true
//     eligibility is unknown) could still beat the winner,
//   * the winner's bisector is nearly parallel to the ray, or it has no hit.
// Node rows rounded from exact FP64 points (node_err > 0) widen the bounds by
// their rounding; the recheck then reads the exact points.
#include "vg_dfloat.h"
#include "vg_internal.h"

namespace vg {
namespace {

constexpr int TILE = kRayTile;

// Scan state of one ray over a range of nodes (t in units of 2t): the
// running top-2 (t, den, node of the best) and the smallest numerator of a
// nearly grazing node.
struct ScanState {
  float t1, t2, den1, den2, gmin;
  int32_t i1;
};

__device__ __forceinline__ ScanState scan_state_empty() {
  return ScanState{__builtin_inff(), __builtin_inff(), 0.f, 0.f, __builtin_inff(), -1};
}

// Folds the state of a later node range into S: equal t keeps S's node, the
// lower index, as the sequential scan does.
__device__ __forceinline__ void scan_state_merge(ScanState &S, const ScanState &T) {
  if (T.t1 < S.t1) {
    S.t2 = S.t1;
    S.den2 = S.den1;
    S.t1 = T.t1;
    S.den1 = T.den1;
    S.i1 = T.i1;
  } else if (T.t1 < S.t2) {
    S.t2 = T.t1;
    S.den2 = T.den1;
  }
  if (T.t2 < S.t2) {
    S.t2 = T.t2;
    S.den2 = T.den2;
  }
  S.gmin = fminf(S.gmin, T.gmin);
}

// One ray's inputs in FP32.
template <int DK>
struct RayIn {
  bool active;
  float x[DK], u[DK], g[DK], gx[DK];
  float rho2;
};

template <int DK>
__device__ __forceinline__ void ray_load(const RayScanArgs &a, int64_t ray, RayIn<DK> &R) {
  const int d = a.d;
  const int32_t gidx = ray < a.m ? a.gen[ray] : 0;
  const bool active = ray < a.m && gidx >= 0 && gidx < a.n;
  // plain local arrays first, then unconditional copies: keeps every array
  // in registers
  float x[DK], u[DK], g[DK];
  if (active) {
    const float *xg = a.nodes + (int64_t)gidx * d;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {
        x[k] = a.o64 ? (float)a.o64[ray * d + k] : a.o32[ray * d + k];
        u[k] = a.u64 ? (float)a.u64[ray * d + k] : a.u32[ray * d + k];
        g[k] = xg[k];
      } else {
        x[k] = u[k] = g[k] = 0.f;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < DK; ++k) x[k] = u[k] = g[k] = 0.f;
  }
  float rho2 = 0.f;
  R.active = active;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    const float e = g[k] - x[k];
    rho2 = __builtin_fmaf(e, e, rho2);
    R.x[k] = x[k];
    R.u[k] = u[k];
    R.g[k] = g[k];
    R.gx[k] = e;
  }
  R.rho2 = rho2;
}

// An invalid generator index is reported and the ray skipped.
__device__ __forceinline__ void report_invalid_gen(const RayScanArgs &a, int64_t ray) {
  if (ray >= a.m) return;
  const int32_t gidx = a.gen[ray];
  if (gidx < 0 || gidx >= a.n) {
    a.t_out[ray] = __builtin_nanf("");
    a.idx_out[ray] = -1;
    a.st_out[ray] = VG_ST_SUSPECT;
  }
}

// grazing test: den^2 <= kd^2 |r - g|^2 with |r - g|^2 <= 2 num + 4 rho^2.
// Node rows rounded from exact points (error up to ne each) move den by up
// to 2 ne: |den| <= kd |r-g| + 2 ne, squared below 2 kd^2 |r-g|^2 + 8 ne^2.
struct GrazeBound {
  float kd2g, ne8;
};
__device__ __forceinline__ GrazeBound graze_bound(const RayScanArgs &a) {
  const float kd = (4.f * (float)(a.d + 4)) * 0x1p-24f;
  const float kd2 = kd * kd;
  const float ne = a.node_err;
  return GrazeBound{ne > 0.f ? 2.f * kd2 : kd2, 8.f * ne * ne};
}

// Nodes [lo, hi) into S; every thread of the workgroup calls it with the
// same range (it contains barriers); sx holds TILE*DK floats.
template <int DK>
__device__ __forceinline__ void ray_scan_nodes(const RayScanArgs &a, int64_t ray, const RayIn<DK> &R, int64_t lo,
                                               int64_t hi, float *sx, ScanState &S) {
  const int tid = threadIdx.x;
  const int d = a.d;
  const GrazeBound gb = graze_bound(a);
  const float rho4 = 4.f * R.rho2;
  float x[DK], u[DK], g[DK], gx[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    x[k] = R.x[k];
    u[k] = R.u[k];
    g[k] = R.g[k];
    gx[k] = R.gx[k];
  }
  // exclusions (sorted) walked alongside the ascending node index from lo
  const int32_t *ex = (R.active && a.n_excl > 0) ? a.excl + ray * a.n_excl : nullptr;
  int ep = 0;
  if (ex)
    while (ep < a.n_excl && (int64_t)ex[ep] < lo) ++ep;
  int32_t next_ex = (ex && ep < a.n_excl) ? ex[ep] : -1;
  float t1 = S.t1, t2 = S.t2, den1 = S.den1, den2 = S.den2, gmin = S.gmin;
  int32_t i1 = S.i1;
  for (int64_t base = lo; base < hi; base += TILE) {
    __syncthreads();
    {
      const int64_t r = base + tid;
#pragma unroll
      for (int k = 0; k < DK; ++k) sx[tid * DK + k] = (r < hi && k < d) ? a.nodes[r * d + k] : 0.f;
    }
    __syncthreads();
    if (!R.active) continue;
    const int cnt = (int)((hi - base) < TILE ? (hi - base) : TILE);
    for (int q = 0; q < cnt; ++q) {
      const int32_t r = (int32_t)(base + q);
      float num = 0.f, den = 0.f;
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        const float xr = sx[q * DK + k];
        const float a_k = xr - g[k];
        num = __builtin_fmaf(a_k, (xr - x[k]) + gx[k], num);
        den = __builtin_fmaf(u[k], a_k, den);
      }
      if (r == next_ex) {
        ++ep;
        next_ex = ep < a.n_excl ? ex[ep] : -1;
        continue;
      }
      if (den * den <= gb.kd2g * __builtin_fmaf(2.f, num, rho4) + gb.ne8) gmin = fminf(gmin, num);
      if (den > 0.f && num < t2 * den) {
        const float t = num / den;
        if (t < t1) {
          t2 = t1;
          den2 = den1;
          t1 = t;
          den1 = den;
          i1 = r;
        } else {
          t2 = t;
          den2 = den;
        }
      }
    }
  }
  S = ScanState{t1, t2, den1, den2, gmin, i1};
}

// Certificate and outputs of an active ray from its full scan state.
template <int DK>
__device__ __forceinline__ void ray_finish(const RayScanArgs &a, int64_t ray, const RayIn<DK> &R,
                                           const ScanState &S) {
  const int d = a.d;
  float x[DK], u[DK], g[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    x[k] = R.x[k];
    u[k] = R.u[k];
    g[k] = R.g[k];
  }
  const float rho2 = R.rho2;
  const float rho4 = 4.f * rho2;
  const GrazeBound gb = graze_bound(a);
  const float kd2g = gb.kd2g, ne8 = gb.ne8, ne = a.node_err;
  const float t1 = S.t1, t2 = S.t2, den1 = S.den1, den2 = S.den2, gmin = S.gmin;
  const int32_t i1 = S.i1;

  // FP32 error bound of t' = num/den for a candidate (units of 2t), u = 2^-24:
  // num = sum_k a_k b_k with a_k = fl(r_k - g_k) (relative error u) and
  // b_k = fl(fl(r_k - x_k) + fl(g_k - x_k)) (off by at most 3u c_k, where
  // c_k = |r_k - x_k| + |g_k - x_k| and |c| <= |r - x| + rho), summed by a
  // chain of d FMAs (gamma_d sum |a_k b_k|): |dnum| <= (d + 4) u |r - g|
  // (|r - x| + rho); den = sum_k u_k a_k likewise: |dden| <= (d + 1) u |r - g|.
  // With rg = |r - x| + rho >= |r - g| (|r - x|^2 = t' den + rho^2), both fit
  // under kap rg^2 and kap rg for kap = 2 (d + 4) u, twice the first-order
  // bound (which also covers the rounding of the division).  An origin
  // rounded from FP64 moves num by up to 2 |r - g| |dx| and a rounded
  // direction moves den by |r - g| |du|.
  const float kap = (2.f * (float)(d + 4)) * 0x1p-24f;
  float xn2 = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) xn2 = __builtin_fmaf(x[k], x[k], xn2);
  const bool rounded = a.o64 != nullptr;
  const float rho = sqrtf(rho2);
  auto tbound = [&](float tc, float dc) {
    const float rx2 = tc * dc + rho2;
    const float rg = sqrtf(fmaxf(rx2, 0.f)) + rho;  // bounds |r - g| and |(r-x)+(g-x)|
    float en = kap * rg * rg;
    float ed = kap * rg;
    if (rounded) {
      en += 2.f * rg * 0x1p-24f * sqrtf(xn2);
      ed += rg * 0x1p-24f;
    }
    if (ne > 0.f) {  // rounded rows of r and g
      en += 2.f * rg * ne;
      ed += 2.f * ne;
    }
    return (en + tc * ed) / dc;
  };
  float eb = 0.f, eb1 = 0.f;
  if (i1 >= 0) eb += eb1 = 0.5f * tbound(t1, den1);
  if (i1 >= 0 && t2 < __builtin_inff()) eb += 0.5f * tbound(t2, den2);
  // a nearly grazing node with true den up to 2 kd |r-g| beats t1' when
  // num < 2 kd |r-g| t1'; in squares: num^2 <= 4 kd^2 (2 num + 4 rho^2) t1'^2
  bool grazing = false;
  if (gmin < __builtin_inff()) {
    grazing = gmin < 0.f ||
              gmin * gmin <= (4.f * kd2g * __builtin_fmaf(2.f, gmin, rho4) + 4.f * ne8) * t1 * t1 ||
              i1 < 0;
  }

  float T1 = 0.5f * t1, T2 = 0.5f * t2;
  int32_t j = i1;
  if (a.clip) {
    float tb = __builtin_inff();
    int face = -1;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d && u[k] != 0.f) {
        const float h = u[k] > 0.f ? 1.f - x[k] : -x[k];
        const float tk = h / u[k];
        if (tk < tb) {
          tb = tk;
          face = 2 * k + (u[k] > 0.f ? 1 : 0);
        }
      }
    }
    if (face >= 0) {
      if (tb < T1) {
        T2 = T1;
        T1 = tb;
        j = -2 - face;
      } else if (tb < T2) {
        T2 = tb;
      }
    }
  }
  uint8_t st = 0;
  bool flag = a.force_all || grazing || !(T2 - T1 > fmaxf(a.tau * T1, 4.f * eb)) ||
              !(4.f * eb1 <= a.tau * T1);
  float t = T1;
  if (j >= 0) {
    // re-evaluate the winner in double-float; check it is not grazing
    const float *xr = a.nodes + (int64_t)j * d;
    dfacc num, den;
    float nrg = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {
        float ah, al, bh, bl, ch, cl;
        two_sum(xr[k], -x[k], ah, al);
        two_sum(g[k], -x[k], bh, bl);
        two_sum(xr[k], -g[k], ch, cl);
        num.add_prod(ah, ah);
        num.add_small(2.f * ah * al);
        num.sub_prod(bh, bh);
        num.add_small(-2.f * bh * bl);
        den.add_prod(u[k], ch);
        den.add_small(u[k] * cl);
        nrg = __builtin_fmaf(ch, ch, nrg);
      }
    }
    float dh, dl;
    den.norm(dh, dl);
    float nu2 = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) nu2 = __builtin_fmaf(u[k], u[k], nu2);
    if (!(dh > (1.f / 4096.f) * sqrtf(nu2 * nrg))) {
      st |= VG_ST_SUSPECT;
      flag = true;
    }
    t = df_half_ratio(num, den);
  } else if (j == -1) {
    st |= VG_ST_NO_HIT;
    t = __builtin_inff();
    flag = true;
  }
  if (flag && a.flag_list) {
    st |= VG_ST_NEAR_TIE;
    const uint32_t pos = atomicAdd(&a.counters[CNT_FLAGGED], 1u);
    a.flag_list[pos] = ray | a.flag_tag;
  }
  a.t_out[ray] = t;
  a.idx_out[ray] = j;
  a.st_out[ray] = st;
}

// Rays [blk*TILE, blk*TILE + TILE) of one problem over all nodes; sx holds
// TILE*DK floats.  Every thread of the workgroup must call it (barriers).
template <int DK>
__device__ __forceinline__ void ray_scan_tile(const RayScanArgs &a, int64_t blk, float *sx) {
  const int64_t ray = blk * TILE + threadIdx.x;
  report_invalid_gen(a, ray);
  RayIn<DK> R;
  ray_load<DK>(a, ray, R);
  ScanState S = scan_state_empty();
  ray_scan_nodes<DK>(a, ray, R, 0, a.n, sx, S);
  if (R.active) ray_finish<DK>(a, ray, R, S);
}

template <int DK>
__global__ __launch_bounds__(TILE) void ray_scan_kernel(RayScanArgs a) {
  __shared__ float sx[TILE * DK];
  ray_scan_tile<DK>(a, blockIdx.x, sx);
}

// Few rays: workgroup (ray tile x, node part y) scans nodes
// [y chunk, (y+1) chunk) and stores its state in parts[y][ray].
template <int DK>
__global__ __launch_bounds__(TILE) void ray_scan_part_kernel(RayScanArgs a, int64_t chunk,
                                                             ScanState *__restrict__ parts) {
  __shared__ float sx[TILE * DK];
  const int64_t ray = (int64_t)blockIdx.x * TILE + threadIdx.x;
  RayIn<DK> R;
  ray_load<DK>(a, ray, R);
  const int64_t lo = (int64_t)blockIdx.y * chunk;
  const int64_t hi = lo + chunk < a.n ? lo + chunk : a.n;
  ScanState S = scan_state_empty();
  ray_scan_nodes<DK>(a, ray, R, lo, hi, sx, S);
  if (ray < a.m) parts[(int64_t)blockIdx.y * a.m + ray] = S;
}

// Folds the parts of each ray in node order, then certifies it as the
// whole-range scan does.
template <int DK>
__global__ __launch_bounds__(TILE) void ray_merge_kernel(RayScanArgs a, int P, const ScanState *__restrict__ parts) {
  const int64_t ray = (int64_t)blockIdx.x * TILE + threadIdx.x;
  if (ray >= a.m) return;
  report_invalid_gen(a, ray);
  RayIn<DK> R;
  ray_load<DK>(a, ray, R);
  if (!R.active) return;
  ScanState S = parts[ray];
  for (int p = 1; p < P; ++p) scan_state_merge(S, parts[(int64_t)p * a.m + ray]);
  ray_finish<DK>(a, ray, R, S);
}

// Node parts of a call with few rays (1: no split): enough workgroups to
// fill the GPU, each part at least two node tiles.
int split_parts(int64_t m, int64_t n) {
  const int64_t tiles = (m + TILE - 1) / TILE;
  if (tiles >= 1024) return 1;
  int64_t P = (2048 + tiles - 1) / tiles;
  const int64_t by_nodes = n / (2 * TILE);
  if (P > by_nodes) P = by_nodes;
  if (P > 256) P = 256;
  return P > 1 ? (int)P : 1;
}

// Uneven batches of problems: workgroups take (problem, ray tile) items from
// a device counter in the order of the item table until it passes the end.
__global__ __launch_bounds__(TILE) void ray_scan_batched_kernel(const RayBatchProblem *probs, int np,
                                                                int64_t total,
                                                                unsigned long long *next) {
  __shared__ float sx[TILE * VG_MAX_DIM];
  __shared__ long long item_s;
  for (;;) {
    __syncthreads();  // the previous item is finished
    if (threadIdx.x == 0) item_s = (long long)atomicAdd(next, 1ull);
    __syncthreads();
    const long long item = item_s;
    if (item >= total) break;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].item_begin <= item)
        lo = mid;
      else
        hi = mid - 1;
    }
    const RayScanArgs a = probs[lo].a;
    const int64_t blk = item - probs[lo].item_begin;
    if (a.d <= 4)
      ray_scan_tile<4>(a, blk, sx);
    else if (a.d <= 8)
      ray_scan_tile<8>(a, blk, sx);
    else if (a.d <= 12)
      ray_scan_tile<12>(a, blk, sx);
    else
      ray_scan_tile<16>(a, blk, sx);
  }
}

}  // namespace

size_t ray_scan_split_bytes(int64_t m, int64_t n) {
  const int P = split_parts(m, n);
  return P > 1 ? (size_t)P * (size_t)m * sizeof(ScanState) : 0;
}

hipError_t launch_ray_scan(const RayScanArgs &a, void *split, size_t split_bytes, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  const int64_t grid64 = (a.m + TILE - 1) / TILE;
  if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid64), blk(TILE);
  const int P = split_parts(a.m, a.n);
  if (P > 1 && split && split_bytes >= (size_t)P * (size_t)a.m * sizeof(ScanState)) {
    const int64_t chunk = ((a.n + P - 1) / P + TILE - 1) / TILE * TILE;
    const int parts = (int)((a.n + chunk - 1) / chunk);
    ScanState *st = static_cast<ScanState *>(split);
    dim3 gsplit((unsigned)grid64, (unsigned)parts);
#define VG_SPLIT(DKV)                                                                       \
  do {                                                                                      \
    hipLaunchKernelGGL(ray_scan_part_kernel<DKV>, gsplit, blk, 0, s, a, chunk, st);         \
    hipLaunchKernelGGL(ray_merge_kernel<DKV>, grid, blk, 0, s, a, parts, (const ScanState *)st); \
  } while (0)
    if (a.d <= 2)
      VG_SPLIT(2);
    else if (a.d <= 3)
      VG_SPLIT(3);
    else if (a.d <= 4)
      VG_SPLIT(4);
    else if (a.d <= 6)
      VG_SPLIT(6);
    else if (a.d <= 8)
      VG_SPLIT(8);
    else if (a.d <= 12)
      VG_SPLIT(12);
    else
      VG_SPLIT(16);
#undef VG_SPLIT
    return hipGetLastError();
  }
  // DK: d rounded up to 2, 3, 4, 6, 8, 12 or 16 (padded coordinates are zeros
  // and add exact zeros to every sum, so the width does not change a result)
  if (a.d <= 2)
    hipLaunchKernelGGL(ray_scan_kernel<2>, grid, blk, 0, s, a);
  else if (a.d <= 3)
    hipLaunchKernelGGL(ray_scan_kernel<3>, grid, blk, 0, s, a);
  else if (a.d <= 4)
    hipLaunchKernelGGL(ray_scan_kernel<4>, grid, blk, 0, s, a);
  else if (a.d <= 6)
    hipLaunchKernelGGL(ray_scan_kernel<6>, grid, blk, 0, s, a);
  else if (a.d <= 8)
    hipLaunchKernelGGL(ray_scan_kernel<8>, grid, blk, 0, s, a);
  else if (a.d <= 12)
    hipLaunchKernelGGL(ray_scan_kernel<12>, grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL(ray_scan_kernel<16>, grid, blk, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ray_scan_batched(const RayBatchProblem *probs_dev, int np, int64_t total,
                                   unsigned long long *next, int grid, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(ray_scan_batched_kernel, dim3(grid), dim3(TILE), 0, s, probs_dev, np, total, next);
  return hipGetLastError();
}

int ray_scan_batched_blocks_per_cu() {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ray_scan_batched_kernel, TILE, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace vg
