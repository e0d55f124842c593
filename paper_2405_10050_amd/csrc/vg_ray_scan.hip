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

// Rays [blk*TILE, blk*TILE + TILE) of one problem; sx holds TILE*DK floats.
// Every thread of the workgroup must call it (it contains barriers).
template <int DK>
__device__ __forceinline__ void ray_scan_tile(const RayScanArgs &a, int64_t blk, float *sx) {
  const int tid = threadIdx.x;
  const int64_t ray = blk * TILE + tid;
  const int d = a.d;
  const int64_t n = a.n;
  int32_t gidx = ray < a.m ? a.gen[ray] : 0;
  if (ray < a.m && (gidx < 0 || gidx >= n)) {  // invalid generator index: report, skip
    a.t_out[ray] = __builtin_nanf("");
    a.idx_out[ray] = -1;
    a.st_out[ray] = VG_ST_SUSPECT;
  }
  const bool active = ray < a.m && gidx >= 0 && gidx < n;

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
  float rho2 = 0.f, gx[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    gx[k] = g[k] - x[k];
    rho2 = __builtin_fmaf(gx[k], gx[k], rho2);
  }
  // grazing test: den^2 <= kd^2 |r - g|^2 with |r - g|^2 <= 2 num + 4 rho^2
  const float kd = (4.f * (float)(d + 4)) * 0x1p-24f;
  const float kd2 = kd * kd;
  // node rows rounded from exact points (error up to ne each) move den by up
  // to 2 ne: |den| <= kd |r-g| + 2 ne, squared below 2 kd^2 |r-g|^2 + 8 ne^2
  const float ne = a.node_err;
  const float kd2g = ne > 0.f ? 2.f * kd2 : kd2;
  const float ne8 = 8.f * ne * ne;
  const float rho4 = 4.f * rho2;
  float gmin = __builtin_inff();  // smallest num of a nearly grazing node
  const int32_t *ex = (active && a.n_excl > 0) ? a.excl + ray * a.n_excl : nullptr;
  int ep = 0;
  int32_t next_ex = ex ? ex[0] : -1;

  float t1 = __builtin_inff(), t2 = __builtin_inff();  // in units of 2t
  float den1 = 0.f, den2 = 0.f;
  int32_t i1 = -1;
  for (int64_t base = 0; base < n; base += TILE) {
    __syncthreads();
    {
      const int64_t r = base + tid;
#pragma unroll
      for (int k = 0; k < DK; ++k) sx[tid * DK + k] = (r < n && k < d) ? a.nodes[r * d + k] : 0.f;
    }
    __syncthreads();
    if (!active) continue;
    const int cnt = (int)((n - base) < TILE ? (n - base) : TILE);
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
      if (den * den <= kd2g * __builtin_fmaf(2.f, num, rho4) + ne8) gmin = fminf(gmin, num);
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
  if (!active) return;

  // FP32 error bound of t' = num/den for a candidate (units of 2t): num and
  // den are sums of d rounded products of differences, |r - x|^2 = t' den +
  // rho^2 and |r - g| <= |r - x| + rho; an origin rounded from FP64 moves num
  // by up to 2 |r - g| |dx| and a rounded direction moves den by |r - g| |du|.
  const float kap = (8.f * (float)(d + 2)) * 0x1p-24f;
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

template <int DK>
__global__ __launch_bounds__(TILE) void ray_scan_kernel(RayScanArgs a) {
  __shared__ float sx[TILE * DK];
  ray_scan_tile<DK>(a, blockIdx.x, sx);
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

hipError_t launch_ray_scan(const RayScanArgs &a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  const int64_t grid64 = (a.m + TILE - 1) / TILE;
  if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid64), blk(TILE);
  if (a.d <= 4)
    hipLaunchKernelGGL(ray_scan_kernel<4>, grid, blk, 0, s, a);
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
