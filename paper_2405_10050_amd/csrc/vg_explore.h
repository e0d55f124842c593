// Internal interface between the exhaustive-search driver and its kernels.
#pragma once

#include "vg_internal.h"

namespace vg {

struct ExploreRays {
  const float *nodes;
  int d;
  int64_t m;               // frontier items
  const int32_t *keys;     // [V][d+1] device vertex keys
  const double *coords;    // [V][d]  device vertex coordinates
  const int64_t *item_v;   // [m] vertex of each item
  const int32_t *item_o;   // [m] position in the key of the omitted generator
  double *o64, *u64;       // [m][d] ray origin and direction (FP64)
  int32_t *gen;            // [m]
  int32_t *excl;           // [m][d] sorted eta
  int32_t *ok;             // [m] direction well defined
  const int32_t *idx;      // [m] raycast result
  int32_t *new_keys;       // [m][d+1] (key[0] < 0: no vertex)
  double *new_coords;      // [m][d]
  int64_t n_nodes;         // nodes (for the sphere check)
};

hipError_t launch_sphere_check(const ExploreRays &a, double *viol, hipStream_t s);

hipError_t launch_edge_rays(const ExploreRays &a, hipStream_t s);
hipError_t launch_new_vertices(const ExploreRays &a, hipStream_t s);
hipError_t launch_descent_project(const float *X, int d, const int32_t *sig, int m, double *u,
                                  int *ok, hipStream_t s);
hipError_t launch_advance(double *r, const double *u, const double *t, int d, double sign,
                          hipStream_t s);
hipError_t launch_solve_one(const float *X, int d, const int32_t *sig, double *v, int *ok,
                            hipStream_t s);

// RayCast of FP64-described rays (FP32 scan, FP64 recheck of flagged rays).
// force_all queues every ray for the FP64 pass; t64 (optional) receives the
// FP64 t of rechecked rays.  Defined in vg_api.hip.
int raycast_f64(vg_ctx *ctx, int d, int64_t n, const float *nodes, int64_t m, const double *o64,
                const double *u64, const int32_t *gen, const int32_t *excl, int n_excl, int clip,
                bool force_all, float *t_out, int32_t *idx_out, uint8_t *st_out, double *t64);

}  // namespace vg
