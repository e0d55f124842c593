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
  int32_t *excl;           // [m][d] kept generators, sorted, padded with INT32_MAX
  int32_t *ok;             // [m] direction well defined
  const int32_t *idx;      // [m] raycast result
  int32_t *new_keys;       // [m][d+1] (key[0] < 0: no vertex)
  double *new_coords;      // [m][d]
  int64_t n_nodes;         // nodes (for the sphere check)
  int32_t face_base;       // clipped diagram: face x_k = s is face_base + 2k + s
                           // in a key; INT32_MAX for the unbounded diagram
};

hipError_t launch_sphere_check(const ExploreRays &a, double *viol, hipStream_t s);

// ---- device bookkeeping of the search (vg_vset.hip)
enum : uint32_t { VSET_FULL = 1, VSET_COLLISION = 2, VSET_SINGULAR = 4 };

// Discovered vertices: slot fingerprint (0 = empty), owner (smallest global
// item index that claimed it; -1 for vertices of earlier levels), key
// [cap][L] with L = d + 1.  cap is a power of two.
struct VSet {
  uint64_t *fp;
  int64_t *owner;
  int32_t *key;
  int64_t cap;
  int L;
};

// Edge visit counts: fingerprint, count, key [cap][d].
struct ESet {
  uint64_t *fp;
  uint32_t *cnt;
  int32_t *key;
  int64_t cap;
};

hipError_t vset_clear(VSet V, hipStream_t s);
hipError_t eset_clear(ESet E, hipStream_t s);
// Insert vertices [0, nv) into V and/or count their edges into E.
hipError_t vset_rebuild(VSet V, ESet E, const int32_t *vkeys, int64_t nv, int d, bool vertices,
                        bool edges, uint32_t *err, hipStream_t s);
// flags[(v - lb)(d+1) + o] = 1 when the edge of vertex v omitting position o
// has been seen fewer than two times (and keeps a generator: entries below
// face_base).
hipError_t frontier_flags(const int32_t *vkeys, int64_t lb, int64_t le, int d, int32_t face_base, ESet E,
                          uint8_t *flags, uint32_t *err, hipStream_t s);
hipError_t frontier_items(const int64_t *sel, int64_t m, int64_t lb, int d, int64_t *item_v,
                          int32_t *item_o, hipStream_t s);
// Claim, settle and verify the new tuples of a level; is_new marks the items
// that own a new vertex, is_unb the items without a hit.
hipError_t vset_insert(VSet V, const int32_t *nkeys, const int32_t *idx, int64_t m, int64_t item_base,
                       int64_t *slot, uint8_t *is_new, uint8_t *is_unb, uint32_t *err, hipStream_t s);
hipError_t append_vertices(const int64_t *sel, int64_t nn, int64_t nv, int d, const int32_t *nkeys,
                           const double *ncoords, int32_t *vkeys, double *vcoords, ESet E, int64_t *eslot,
                           uint32_t *err, hipStream_t s);
hipError_t append_unbounded(const int64_t *sel, int64_t nb, int64_t b0, int d, const int64_t *item_v,
                            const int32_t *item_o, const int32_t *vkeys, int32_t *bsig, int32_t *bomit,
                            hipStream_t s);
hipError_t select_flagged(void *temp, size_t &temp_bytes, const uint8_t *flags, int64_t n, int64_t *out,
                          int64_t *count_dev, hipStream_t s);

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
// FP64 t of rechecked rays; incircle 1 (2) casts by Algorithm 1 without
// (with) InitialHeuristic, counting queries in the context's counters.
// Defined in vg_api.hip.
int raycast_f64(vg_ctx *ctx, int d, int64_t n, const float *nodes, int64_t m, const double *o64,
                const double *u64, const int32_t *gen, const int32_t *excl, int n_excl, int clip,
                bool force_all, float *t_out, int32_t *idx_out, uint8_t *st_out, double *t64,
                int incircle);

}  // namespace vg
