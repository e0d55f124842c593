// Internal interface between the exhaustive-search driver and its kernels.
#pragma once

#include "vg_internal.h"

namespace vg {

// Periodic diagram (the torus R^d / Z^d, Sec. 1): every node x_i in [0,1)^d
// stands for its images x_i + k, k in Z^d.  A key entry is an image coded
// i S + c(k) with S = 3^d and c(k) = sum_a (k_a + 1) 3^a, k in {-1,0,1}^d.
// Rays are cast over the images inside [-w, 1+w]^d (FP32 rows, ordered with
// the k = 0 images first, so image i is node i); vertex coordinates are
// solved from the exact FP64 images.
struct Periodic {
  int32_t S = 0;                  // 3^d; 0 when the diagram is not periodic
  const float *X = nullptr;       // [n][d] the nodes
  const int32_t *tkey = nullptr;  // [n_img] code of each scanned image
  const int32_t *tix = nullptr;   // [n S] scanned image of each code, -1 outside the layer
  int64_t n_codes = 0;            // n S
  double w = 0.0;                 // the layer: images in [-w, 1+w]^d
};

// Digit a of the code c (k_a + 1).
__host__ __device__ inline int code_digit(int32_t c, int a) {
  for (int q = 0; q < a; ++q) c /= 3;
  return c % 3;
}

// Translates the sorted key (L entries i S + c) by a lattice vector so that
// its first entry has k = 0.  False when a node repeats or a shift leaves
// {-1,0,1}^d (then the key is left partly rewritten).
__host__ __device__ inline bool periodic_canon(int32_t *key, int L, int d, int32_t S) {
  const int32_t c0 = key[0] % S;
  for (int e = 0; e < L; ++e) {
    const int32_t id = key[e] / S;
    int32_t c = key[e] % S, r0 = c0, cn = 0, p = 1;
    for (int a = 0; a < d; ++a) {
      const int dig = c % 3 - r0 % 3 + 1;
      if (dig < 0 || dig > 2) return false;
      cn += dig * p;
      p *= 3;
      c /= 3;
      r0 /= 3;
    }
    if (e > 0 && id == key[e - 1] / S) return false;
    key[e] = id * S + cn;
  }
  return true;
}

// Coordinate k of the image coded e, exact in FP64.
__device__ inline double image_coord(const Periodic &P, int d, int32_t e, int k) {
  const int32_t i = e / P.S;
  return (double)P.X[(int64_t)i * d + k] + (double)(code_digit(e % P.S, k) - 1);
}

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
  Periodic per;            // periodic diagram: keys hold image codes, rays run
                           // over the scanned images (nodes, n_nodes)
  uint32_t *err;           // VSET_* error word
};

hipError_t launch_sphere_check(const ExploreRays &a, double *viol, hipStream_t s);

// ---- device bookkeeping of the search (vg_vset.hip)
// VSET_THIN: a periodic vertex ball reaching past the scanned image layer,
// or a periodic ray without a hit (the layer is too thin: widen it);
// VSET_RANGE: a periodic key whose shifts leave {-1,0,1}^d or that holds a
// node twice (a vertex ball of radius >= 1/2).
enum : uint32_t { VSET_FULL = 1, VSET_COLLISION = 2, VSET_SINGULAR = 4, VSET_THIN = 8, VSET_RANGE = 16 };

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

// Edge visit counts: fingerprint, count, key [cap][d].  On the periodic
// diagram (S = 3^d, else 0) an edge key is translated like a vertex key.
struct ESet {
  uint64_t *fp;
  uint32_t *cnt;
  int32_t *key;
  int64_t cap;
  int32_t S;
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
// The vertex of one key: node indices over X, or (per.S > 0) image codes.
hipError_t launch_solve_one(const float *X, int d, const int32_t *sig, const Periodic &per, double *v,
                            int *ok, hipStream_t s);

// RayCast of FP64-described rays (FP32 scan, FP64 recheck of flagged rays).
// force_all queues every ray for the FP64 pass; t64 (optional) receives the
// FP64 t of rechecked rays; incircle 1 (2) casts by Algorithm 1 without
// (with) InitialHeuristic, counting queries in the context's counters.
// nodes64 (optional, dense scan only) holds the exact FP64 points the FP32
// rows were rounded from, each row within node_err of its point: the FP32
// certificate widens by that and the recheck reads the exact points.
// Defined in vg_api.hip.
int raycast_f64(vg_ctx *ctx, int d, int64_t n, const float *nodes, int64_t m, const double *o64,
                const double *u64, const int32_t *gen, const int32_t *excl, int n_excl, int clip,
                bool force_all, float *t_out, int32_t *idx_out, uint8_t *st_out, double *t64,
                int incircle, const double *nodes64 = nullptr, float node_err = 0.f,
                bool check_input = false);

}  // namespace vg
