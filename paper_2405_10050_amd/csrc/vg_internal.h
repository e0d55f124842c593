// Internal declarations of the gfx950 batched RayCast library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vgraph.h"

namespace vg {

// Device-side counters kept in the context (one block of device memory).
enum : int {
  CNT_FLAGGED = 0,   // rays appended to the FP64 recheck list
  CNT_FP64_TIE = 1,  // rays whose FP64 gap is below 1e-9
  CNT_WORDS = 4
};

// Where the recheck kernel finds a ray.
enum RayMode : int { RAYS_CELLS = 0, RAYS_F32 = 1, RAYS_F64 = 2 };

struct RayScanArgs {
  const float *nodes;
  int64_t n;
  int d;
  int64_t m;            // rays
  const float *o32;     // origins f32 [m][d] (mode F32), or null
  const float *u32;
  const double *o64;    // origins f64 [m][d] (mode F64), or null
  const double *u64;
  const int32_t *gen;
  const int32_t *excl;  // [m][n_excl]
  int n_excl;
  int clip;
  float *t_out;
  int32_t *idx_out;
  uint8_t *st_out;      // never null inside the library (scratch if the caller passes null)
  uint32_t *counters;
  int64_t *flag_list;
  float tau;
  int force_all;  // queue every ray for the FP64 recheck
};

struct CellScanArgs {
  const float *nodes;
  int64_t n;
  int d;
  const float *dirs;  // [n][R][d]
  int R;
  int wg_per_cell;
  float *t_out;
  int32_t *idx_out;
  uint8_t *st_out;
  uint32_t *counters;
  int64_t *flag_list;
  float tau_rel;      // relative gap floor
  float kappa;        // absolute FP32 error bound coefficient (times 1/nn-distance)
};

struct RecheckArgs {
  int mode;
  const float *nodes;
  int64_t n;
  int d;
  const float *dirs;  // cells mode
  int R;
  const float *o32, *u32;
  const double *o64, *u64;
  const int32_t *gen, *excl;
  int n_excl;
  int clip;
  const uint32_t *counters;
  const int64_t *flag_list;
  float *t_out;
  int32_t *idx_out;
  uint8_t *st_out;
  uint32_t *tie_counter;
  double *t64_out;  // optional FP64 t of each rechecked ray
};

struct AccumArgs {
  const float *nodes;
  int64_t n;
  int d;
  int R;
  const float *t;
  const int32_t *idx;
  float sv, se, sa;  // scales S/(dn), S/((d+2)n), S/n
  float *volume;
  float *energy2;
  int32_t *facet_j;
  float *facet_area;
  int32_t *facet_count;
};

struct BackwardArgs {
  const float *nodes;
  int64_t n;
  int d;
  int R;
  const float *dirs;
  const float *t;
  const int32_t *idx;
  const int32_t *facet_j;
  const int32_t *facet_count;
  const float *gv, *ge, *ga;
  float sv, se, sa;
  float *own;            // [n][d] own-cell part of the gradient
  float *rec;            // [n][R][d] per-facet contribution to the winner
  int32_t *rec_j;        // [n][R] winner of each record (-1: none)
  uint32_t *maxabs;      // [n] float bits of the largest |record| aimed at j
  uint32_t *count;       // [n] records aimed at j
  unsigned long long *acc;  // [n][d] fixed-point sums
  float *grad;           // [n][d]
};

// Launchers (return a hipError_t of the launch).
hipError_t launch_cell_scan_fp32(const CellScanArgs &a, hipStream_t s);
hipError_t launch_cell_scan_bf16x3(const CellScanArgs &a, hipStream_t s);
hipError_t launch_ray_scan(const RayScanArgs &a, hipStream_t s);
hipError_t launch_recheck(const RecheckArgs &a, int max_grid, hipStream_t s);
hipError_t launch_accum(const AccumArgs &a, hipStream_t s);
hipError_t launch_backward(const BackwardArgs &a, hipStream_t s);
hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

// Cell-scan tile choice: rays per workgroup for a given rays-per-cell.
int cell_scan_rays_per_wg(int R);

// Relative gap floors of the near-tie test.  The cell scan certifies its
// argmax with an absolute FP32/BF16x3 error bound (kappa / nn-distance); the
// floors below only keep a margin of a few ulps on top of it.  General rays
// use a wider floor plus their own per-candidate bound.
constexpr float kTauCellsFp32 = 1.0f / 1048576.0f;  // 2^-20
constexpr float kTauCellsBf16 = 1.0f / 16384.0f;    // 2^-14
constexpr float kTauRays = 1.0f / 1024.0f;          // 2^-10

}  // namespace vg

struct vg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  uint32_t *counters = nullptr;  // device [CNT_WORDS]
  int64_t last_rays = 0;
  double last_tau = 0.0;
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> scan_events;  // pending timings
  int64_t scan_launches = 0;
  double scan_ms = 0.0;
};
