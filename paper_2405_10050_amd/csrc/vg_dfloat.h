// Error-free transformations in FP32 (Knuth's TwoSum, FMA-based TwoProduct;
// Ogita, Rump & Oishi, "Accurate sum and dot product", SIAM J. Sci. Comput.
// 2005) used to re-evaluate the winning t* of a ray to about FP32 rounding,
// without FP64 arithmetic.  Every body turns FP contraction off: fusing the
// product of TwoProduct into the following sum (allowed by the default
// -ffp-contract=fast) silently breaks the transformation.
#pragma once

#include <hip/hip_runtime.h>

namespace vg {

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

// (hi, lo) accumulator of a sum of products.
struct dfacc {
  float s = 0.f, e = 0.f;
  __device__ __forceinline__ void add_prod(float a, float b) {
#pragma clang fp contract(off)
    float p, pe, s2, e2;
    two_prod(a, b, p, pe);
    two_sum(s, p, s2, e2);
    s = s2;
    e += e2 + pe;
  }
  __device__ __forceinline__ void sub_prod(float a, float b) { add_prod(-a, b); }
  __device__ __forceinline__ void add_small(float v) {
#pragma clang fp contract(off)
    e += v;
  }
  __device__ __forceinline__ void norm(float &hi, float &lo) const {
#pragma clang fp contract(off)
    hi = s + e;
    lo = e - (hi - s);
  }
};

// t = num / (2 den) for double-float num and den.
__device__ __forceinline__ float df_half_ratio(const dfacc &num, const dfacc &den) {
#pragma clang fp contract(off)
  float nh, nl, dh, dl;
  num.norm(nh, nl);
  den.norm(dh, dl);
  float q = nh / dh;
  float r = __builtin_fmaf(-q, dh, nh);
  return 0.5f * (q + (r + nl - q * dl) / dh);
}

// t of eq. (t) for a Monte-Carlo ray (origin x_i, direction u) ending on
// the bisector of x_i and node x_j, t = |x_j - x_i|^2 / (2 u.(x_j - x_i)),
// in double-float: x_j - x_i is formed exactly as h + l (TwoSum).
template <int DK>
__device__ float reeval_cell(const float (&xi)[DK], const float *__restrict__ xj,
                             const float (&u)[DK], int d) {
  dfacc num, den;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    if (k < d) {
      float h, l;
      two_sum(xj[k], -xi[k], h, l);  // x_j - x_i exactly as h + l
      num.add_prod(h, h);
      num.add_small(2.f * h * l);
      den.add_prod(u[k], h);
      den.add_small(u[k] * l);
    }
  }
  return df_half_ratio(num, den);
}

}  // namespace vg
