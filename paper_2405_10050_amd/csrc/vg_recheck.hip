// FP64 re-evaluation of the rays whose FP32 scan could not certify its
// argmin (near-ties, no hit, grazing winners).
//
// For each queued ray a workgroup scans every node in FP64 with eq. (t) in
// difference form, t = (|r - x|^2 - |g - x|^2) / (2 u.(r - g)) over nodes
// with u.(r - g) > 0 not in eta, keeps the smallest t (lowest index on
// equality), applies the cube clip, and overwrites the ray's result.  The
// list length is read on the device, so the launch needs no host sync: a
// fixed grid strides over the list.  FP contraction is off here so that each
// t is the same IEEE expression as a plain sequential evaluation.
#include "vg_internal.h"

namespace vg {
namespace {

constexpr int NT = 256;

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

#pragma clang fp contract(off)
__global__ __launch_bounds__(NT) void recheck_kernel(RecheckArgs a) {
  __shared__ double sx[VG_MAX_DIM], su[VG_MAX_DIM], sg[VG_MAX_DIM];
  __shared__ int32_t sex[VG_MAX_DIM];
  __shared__ double rt1[NT], rt2[NT];
  __shared__ int32_t ri1[NT];
  const int tid = threadIdx.x;
  const int d = a.d;
  const uint32_t cnt = a.counters[CNT_FLAGGED];
  for (uint32_t f = blockIdx.x; f < cnt; f += gridDim.x) {
    const int64_t ray = a.flag_list[f];
    int n_excl = 0;
    int32_t gi;
    int clip;
    if (a.mode == RAYS_CELLS) {
      const int64_t cell = ray / a.R;
      gi = (int32_t)cell;
      n_excl = 1;
      clip = 1;
      if (tid < d) {
        sx[tid] = (double)a.nodes[cell * d + tid];
        su[tid] = (double)a.dirs[ray * d + tid];
      }
      if (tid == 0) sex[0] = gi;
    } else {
      gi = a.gen[ray];
      n_excl = a.n_excl;
      clip = a.clip;
      if (tid < d) {
        sx[tid] = a.mode == RAYS_F64 ? a.o64[ray * d + tid] : (double)a.o32[ray * d + tid];
        su[tid] = a.mode == RAYS_F64 ? a.u64[ray * d + tid] : (double)a.u32[ray * d + tid];
      }
      if (tid < n_excl) sex[tid] = a.excl[ray * n_excl + tid];
    }
    if (tid < d) sg[tid] = (double)a.nodes[(int64_t)gi * d + tid];
    __syncthreads();
    double rho2 = 0.0;
    for (int k = 0; k < d; ++k) {
      const double e = sg[k] - sx[k];
      rho2 += e * e;
    }
    Top2 tp{__builtin_inf(), __builtin_inf(), -1};
    for (int64_t r = tid; r < a.n; r += NT) {
      bool skip = false;
      for (int q = 0; q < n_excl; ++q) skip |= (sex[q] == (int32_t)r);
      if (skip) continue;
      const float *xr = a.nodes + r * d;
      double den = 0.0;
      for (int k = 0; k < d; ++k) den += su[k] * ((double)xr[k] - sg[k]);
      if (!(den > 0.0)) continue;
      double num = 0.0;
      for (int k = 0; k < d; ++k) {
        const double e = (double)xr[k] - sx[k];
        num += e * e;
      }
      num -= rho2;
      const double t = num / (2.0 * den);
      if (t < tp.t1) {
        tp.t2 = tp.t1;
        tp.t1 = t;
        tp.i1 = (int32_t)r;
      } else if (t < tp.t2) {
        tp.t2 = t;
      }
    }
    rt1[tid] = tp.t1;
    rt2[tid] = tp.t2;
    ri1[tid] = tp.i1;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        Top2 x{rt1[tid], rt2[tid], ri1[tid]}, y{rt1[tid + s], rt2[tid + s], ri1[tid + s]};
        Top2 z = merge(x, y);
        rt1[tid] = z.t1;
        rt2[tid] = z.t2;
        ri1[tid] = z.i1;
      }
      __syncthreads();
    }
    if (tid == 0) {
      double t1 = rt1[0], t2 = rt2[0];
      int32_t i1 = ri1[0];
      if (clip) {
        double tb = __builtin_inf();
        int face = -1;
        for (int k = 0; k < d; ++k) {
          double tk;
          int fc;
          if (su[k] > 0.0) {
            tk = (1.0 - sx[k]) / su[k];
            fc = 2 * k + 1;
          } else if (su[k] < 0.0) {
            tk = (0.0 - sx[k]) / su[k];
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
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_recheck(const RecheckArgs &a, int max_grid, hipStream_t s) {
  if (max_grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(recheck_kernel, dim3(max_grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace vg
