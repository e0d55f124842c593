// Monte-Carlo directions drawn on the device (Sec. 3.1: u uniform on the unit
// sphere, drawn in Algorithm 3 as a normalised standard normal vector).
//
// Generator: Philox4x32-10, the counter-based generator of Salmon, Moraes,
// Dror and Shaw (SC'11): ten rounds of two 32x32->64-bit products with the
// multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by 0x9E3779B9 and
// 0xBB67AE85 between rounds.  Each call maps a 128-bit counter and a 64-bit
// key to four 32-bit words; nothing is stored between calls, so any ray's
// direction is a pure function of (seed, cell, ray) and every kernel that
// needs it recomputes it where it is used.
//
// Direction k-th component of ray `ray` of cell `cell`:
//   call j = k / 4 with counter (j, ray, cell mod 2^32, cell / 2^32) and key
//   (seed mod 2^32, seed / 2^32) gives words w0..w3; pair p = (k mod 4) / 2
//   uses a = w_{2p}, b = w_{2p+1}:
//     u1 = (a + 1/2) 2^-32 in (0, 1),  u2 = b 2^-32 in [0, 1),
//     rho = sqrt(-2 ln u1),  theta = 2 pi u2   (Box-Muller, in FP64),
//     z_k = rho cos theta (k even), rho sin theta (k odd);
//   s = z_0^2 + z_1^2 + ... (in this order, no fused multiply-add),
//   u_k = fp32(z_k / sqrt(s)).
// The rounded vector is used as given (it is not renormalised in FP32).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vg {

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Direction of Monte-Carlo ray `ray` of cell `cell` (components d..DK-1 zero).
template <int DK>
__device__ __forceinline__ void mc_direction(uint64_t seed, int64_t cell, int ray, int d, float (&u)[DK]) {
#pragma clang fp contract(off)
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  double z[DK];
#pragma unroll
  for (int j = 0; j < (DK + 3) / 4; ++j) {
    uint32_t c[4] = {(uint32_t)j, (uint32_t)ray, (uint32_t)(uint64_t)cell, (uint32_t)((uint64_t)cell >> 32)};
    if (4 * j < d) philox4x32_10(c, k0, k1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int k = 4 * j + 2 * p;
      if (k < DK) {
        double zc = 0.0, zs = 0.0;
        if (k < d) {
          const double u1 = ((double)c[2 * p] + 0.5) * 0x1p-32;
          const double u2 = (double)c[2 * p + 1] * 0x1p-32;
          const double rho = sqrt(-2.0 * log(u1));
          double sn, cs;
          sincos(6.283185307179586 * u2, &sn, &cs);
          zc = rho * cs;
          zs = rho * sn;
        }
        z[k] = zc;
        if (k + 1 < DK) z[k + 1] = zs;
      }
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < DK; ++k)
    if (k < d) s = s + z[k] * z[k];
  const double q = sqrt(s);
#pragma unroll
  for (int k = 0; k < DK; ++k) u[k] = k < d ? (float)(z[k] / q) : 0.f;
}

// Direction of ray `ray` of `cell`: read from dirs [n][R][d] when given, else
// drawn from `seed`; zero for ray >= R.
template <int DK>
__device__ __forceinline__ void cell_dir(const float *__restrict__ dirs, uint64_t seed, int64_t cell, int R,
                                         int ray, int d, float (&u)[DK]) {
  if (ray >= R) {
#pragma unroll
    for (int k = 0; k < DK; ++k) u[k] = 0.f;
  } else if (dirs) {
    const float *up = dirs + ((int64_t)cell * R + ray) * d;
#pragma unroll
    for (int k = 0; k < DK; ++k) u[k] = k < d ? up[k] : 0.f;
  } else {
    mc_direction<DK>(seed, cell, ray, d, u);
  }
}

}  // namespace vg
