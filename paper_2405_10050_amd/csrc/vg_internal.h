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
  CNT_BAD_NODES = 2, // non-finite node coordinates seen by the call's input check
  CNT_BAD_RAYS = 3,  // rays answered NaN / -1 because of non-finite input
  CNT_NN_CALLS = 4,  // u64 (words 4, 5): nearest-neighbour queries of the incircle RayCast
  CNT_NN_GRID = 6,   // u64 (words 6, 7): of those, queries answered by the grid
  CNT_SCAN_BLOCKS = 8,  // u64 (words 8, 9): 32x32 MFMA blocks the Monte-Carlo scan evaluated
  CNT_WORDS = 10
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
  int force_all;     // queue every ray for the FP64 recheck
  int64_t flag_tag;  // ORed into queued ray ids (batched mode: problem << 40)
  float node_err;    // bound on |row - exact point| of a node row (rows rounded
                     // from FP64 points, e.g. periodic images); 0: rows exact
};

// One problem of a persistent batch of general rays: its scan arguments and
// the first global item (256-ray tile) of its rays.
struct RayBatchProblem {
  RayScanArgs a;
  int64_t item_begin;
};

struct CellScanArgs {
  const float *nodes;
  int64_t n;
  int d;
  const float *dirs;  // [n][R][d], or null: drawn from `seed` (vg_philox.h)
  uint64_t seed;
  int R;
  int wg_per_cell;
  float *t_out;
  int32_t *idx_out;
  uint8_t *st_out;
  uint32_t *counters;
  int64_t *flag_list;
  float tau_rel;      // relative gap floor
  float kappa;        // absolute FP32 error bound coefficient (times 1/nn-distance)
  int64_t flag_tag;   // ORed into queued ray ids (batched mode: problem << 40)
  // optional candidate lists (CSR): cell i scans only nodes nbr[nbr_off[i] ..
  // nbr_off[i+1]); null scans every node
  const int64_t *nbr_off;
  const int32_t *nbr;
  // optional scan order (no candidate lists): xs[p] = node perm[p], and
  // rank[i] is the position of node i; the scan then starts at the cell's
  // own position and skips blocks that cannot reach a lane's second best
  const float *xs;
  const int32_t *perm;
  const int32_t *rank;
  const float *aabb;  // per kOrderGroup nodes of xs: boxes, then balls (order_box_floats)
};

// One cloud of a persistent batch: its scan arguments and the first global
// item of its (cell, ray-chunk) items.
struct BatchProblem {
  CellScanArgs a;
  int64_t item_begin;
};

struct RecheckArgs {
  int mode;
  const float *nodes;
  int64_t n;
  int d;
  const float *dirs;  // cells mode ([n][R][d], or null: drawn from `seed`)
  uint64_t seed;
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
  const double *nodes64;  // RAYS_F64: exact FP64 node rows read in place of
                          // `nodes` when set (rows rounded for the FP32 scan)
};

struct AccumArgs {
  const float *nodes;
  int64_t n;
  int d;
  int R;
  const float *t;
  const int32_t *idx;
  float sv, se, sa;  // scales S/(dn), S/((d+2)n), S/n
  float *volume;      // or null
  float *energy2;     // or null
  int32_t *facet_j;   // facet rows (null: no facets)
  float *facet_area;  // or null
  int32_t *facet_count;
  // integrals of a function f (Algorithm 3's F_V and F), when fvals is set
  int m;                // draws per ray for the volume integral (0: none)
  const float *tsamp;   // [n][R][m] draws t in (0, 1)
  const float *fvals;   // [n][R][m+1]: f at the hit point, then at the m interior points
  float sf;             // S/(n m)
  float *fint_volume;   // [n] or null
  float *fint_facet;    // [n][R], aligned with facet_j, or null
};

struct BackwardArgs {
  const float *nodes;
  int64_t n;
  int d;
  int R;
  const float *dirs;  // [n][R][d], or null: drawn from `seed`
  uint64_t seed;
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

// Scan order of the nodes (vg_order.hip): sort keys needed for n nodes (a
// power of two >= n), and the pass that fills perm, rank, xs and, per group
// of kOrderGroup consecutive nodes of xs, the bounding box and a bounding
// ball (aabb: G = ceil(n / kOrderGroup) boxes of 2d floats, d minima then d
// maxima, followed by G balls of d + 1 floats, the centre then a radius that
// holds every node of the group; order_box_floats floats in all).
constexpr int kOrderGroup = 128;
__host__ __device__ inline int64_t order_groups(int64_t n) { return (n + kOrderGroup - 1) / kOrderGroup; }
__host__ __device__ inline int64_t order_box_floats(int64_t n, int d) { return order_groups(n) * (3 * (int64_t)d + 1); }
// Whether a Monte-Carlo scan of dimension d runs in scan order: the flags
// decide, else d <= 12 for FP32 and d <= 10 for BF16x3 (measured on uniform
// clouds at 256 rays per cell: beyond, nearly every block is evaluated and
// the order's bookkeeping costs more than it saves; FP32 d=12: 272 ms in scan
// order against 331 ms, d=16: 496 against 439; BF16x3 d=12: 158 against 139).
inline bool scan_order(int d, uint32_t flags, bool bf16) {
  if (flags & VG_INDEX_ORDER) return false;
  return (flags & VG_SCAN_ORDER) || d <= (bf16 ? 10 : 12);
}
int64_t node_order_keys(int64_t n);
hipError_t launch_node_order(const float *nodes, int64_t n, int d, uint64_t *keys, int32_t *perm, int32_t *rank,
                             float *xs, float *aabb, hipStream_t s);
// The Monte-Carlo cell scan over cells [0, grid / a.wg_per_cell): one
// translation unit per (directions drawn, nodes in scan order) instance set.
hipError_t launch_cells_read_index(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s);
hipError_t launch_cells_read_sorted(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s);
hipError_t launch_cells_gen_index(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s);
hipError_t launch_cells_gen_sorted(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s);

// Launchers (return a hipError_t of the launch).
hipError_t launch_cell_scan_fp32(const CellScanArgs &a, hipStream_t s);
hipError_t launch_cell_scan_bf16x3(const CellScanArgs &a, hipStream_t s);
// The same over cells [0, n_cells) with rw rays per workgroup (64, 128, 256,
// 512 or 1024; a.wg_per_cell is set from it).
hipError_t launch_cell_scan_rw(const CellScanArgs &a, bool bf16, int rw, int64_t n_cells, hipStream_t s);
// Directed generator adjacency (CSR) of a set of vertex tuples; synchronises
// the stream.  Defined in vg_nbr.hip.
int tuple_neighbors(int d, int64_t n_nodes, int64_t n_tuples, const int32_t *sigma,
                    int64_t *offsets, int32_t *nbr, int64_t nbr_capacity, int64_t *nnz_out,
                    hipStream_t s, std::string &err);

// Heuristic Monte-Carlo integrals (Sec. 3.3) over a clipped vertex set
// (vg_hmc.hip): the centroid pass (integrals false) or the integral pass.
int hmc_run(bool integrals, int d, int64_t n, const float *nodes, int64_t V, const int32_t *sigma,
            const double *coords, const float *fv, int R, const int32_t *facet_j, const float *facet_area,
            const int32_t *facet_count, const float *fc, const float *fx, float *centroid, int32_t *kcount,
            float *F, float *cell, float *volume, hipStream_t s, std::string &err);

// Incircle RayCast (Algorithm 1) of the Monte-Carlo rays with a grid index
// (vg_incircle.hip): scratch of incircle_scratch_bytes(n, d, R); query counts
// added to nn_calls[0] (all) and nn_calls[1] (answered by the grid).
size_t incircle_scratch_bytes(int64_t n, int d, int R);
hipError_t launch_incircle_cells(const CellScanArgs &a, void *scratch, unsigned long long *nn_calls,
                                 hipStream_t s);
// The same for general rays (scratch of incircle_rays_scratch_bytes; query
// counts added to nn_calls[0] and nn_calls[1]); heuristic applies
// InitialHeuristic to rays with |eta| >= 2.
size_t incircle_rays_scratch_bytes(int64_t n, int d);
hipError_t launch_incircle_rays(const RayScanArgs &a, void *scratch, int heuristic, unsigned long long *nn_calls,
                                hipStream_t s);

// split: device scratch of ray_scan_split_bytes(m, n) bytes (or null): a call
// with few rays then splits the node range over workgroups and merges.
size_t ray_scan_split_bytes(int64_t m, int64_t n);
hipError_t launch_ray_scan(const RayScanArgs &a, void *split, size_t split_bytes, hipStream_t s);
constexpr int kRayTile = 256;  // rays per workgroup (and per batched item) of the ray scan
hipError_t launch_ray_scan_batched(const RayBatchProblem *probs_dev, int np, int64_t total,
                                   unsigned long long *next, int grid, hipStream_t s);
int ray_scan_batched_blocks_per_cu();
hipError_t launch_recheck_rays_batched(const RayBatchProblem *probs_dev, const uint32_t *counters,
                                       const int64_t *flag_list, uint32_t *tie_counter, int grid,
                                       hipStream_t s);
// queued: the queue length when the caller knows it (-1: read on the device only)
hipError_t launch_recheck(const RecheckArgs &a, int max_grid, hipStream_t s, int64_t queued = -1);
// Monte-Carlo rays over n >= 2^18 nodes: the recheck split over node chunks,
// driven by the queue length on the device (m rays at most); parts scratch
// of recheck_cells_reserve(m, n) bytes (0: no split, use launch_recheck).
size_t recheck_cells_reserve(int64_t m, int64_t n);
bool launch_recheck_cells_split(const RecheckArgs &a, int64_t m, void *parts, size_t parts_bytes, hipStream_t s,
                                hipError_t &err);
// General rays with a known queue length cnt (host): where one workgroup
// per queued ray would stream many nodes, split each ray's nodes over
// workgroups and merge.  Returns false (nothing launched) when the split does
// not apply; parts: device scratch of recheck_split_reserve(m, n) bytes.
size_t recheck_split_reserve(int64_t m, int64_t n);
bool launch_recheck_split(const RecheckArgs &a, uint32_t cnt, void *parts, size_t parts_bytes, hipStream_t s,
                          hipError_t &err);
hipError_t launch_accum(const AccumArgs &a, hipStream_t s);
// Sample points of Algorithm 3 per ray: the hit point x_i + l u, then the m
// interior points x_i + t_s l u.  points [n][R][m+1][d].
hipError_t launch_sample_points(const float *nodes, int64_t n, int d, int R, const float *dirs, const float *t,
                                int m, const float *tsamp, float *points, hipStream_t s);
hipError_t launch_backward(const BackwardArgs &a, hipStream_t s);
hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Count the non-finite values of x[0 .. count) into *bad (vg_util.hip).
hipError_t launch_check_finite(const float *x, int64_t count, uint32_t *bad, hipStream_t s);
// After a raycast-type call: every ray gets t = NaN, idx = -1 and
// VG_ST_BAD_INPUT when counters[CNT_BAD_NODES] is set or when its own input
// (its rows of u32, o32, u64, o64, those given) is not finite; counted in
// counters[CNT_BAD_RAYS].
struct FinalizeArgs {
  int64_t m;
  int d;
  const float *o32;  // [m][d] or null
  const float *u32;  // [m][d] or null
  const double *o64;  // [m][d] or null
  const double *u64;  // [m][d] or null
  const uint32_t *flags;  // counters of the call
  uint32_t *bad_rays;
  float *t_out;
  int32_t *idx_out;
  uint8_t *st_out;
};
hipError_t launch_finalize_bad(const FinalizeArgs &f, hipStream_t s);

hipError_t launch_recheck_batched(const BatchProblem *probs_dev, const uint32_t *counters,
                                  const int64_t *flag_list, uint32_t *tie_counter, int grid,
                                  hipStream_t s);

// Error-bound coefficient of the cell scan's near-tie certificate: the
// computed u.r~ of any node is within c |r~| <= c / nn of the exact value, so
// a gap above 2 c / nn certifies the argmax.
//   FP32:    c = (2d + 4) 2^-24   (inverted node (d+4) ulps, K = d products);
//            kappa = 4 (margin) * 2 c.
//   BF16x3:  bf16 keeps 8 significant bits (unit roundoff 2^-8), so
//            a = hi + lo + e with |e| <= 2^-16 |a| and |lo| <= 2^-8 |a|: the
//            dropped lo*lo and the two remainders e_a b, a e_b are at most
//            3 * 2^-16 |a b| (to first order), plus (4d + 4) 2^-24 for the
//            inverted node and the FP32 accumulation of 3d terms;
//            kappa = 2 (3 * 2^-16 + 4 (margin) (4d + 4) 2^-24).  The split
//            term has no margin of its own: the factor 4 on the FP32 term
//            (at least 3 (4d + 4) 2^-24 = 2^-17.4 spare) covers the
//            second-order parts (about 2^-7 * 2^-16) many times over.
inline float cell_kappa(int d, bool bf16) {
  if (bf16) return 2.f * (3.f * 0x1p-16f + 4.f * (4.f * d + 4.f) * 0x1p-24f);
  return 4.f * 2.f * (2.f * d + 4.f) * 0x1p-24f;
}

void batch_state_free(vg_ctx *ctx);

// Device scratch of one Monte-Carlo RayCast call (run_cells_in): the FP64
// recheck queue [m], the status bytes [m], the incircle grid, the node-split
// recheck parts, and the CNT_WORDS counters.
struct CellsScratch {
  // scan order of the nodes (vg_order.hip), or all null: index order
  uint64_t *order_keys = nullptr;  // node_order_keys(n) entries
  int32_t *perm = nullptr, *rank = nullptr;
  float *xs = nullptr, *aabb = nullptr;
  int64_t *flag_list = nullptr;
  uint8_t *status = nullptr;
  void *grid = nullptr;
  void *parts = nullptr;
  size_t parts_bytes = 0;
  uint32_t *counters = nullptr;
  bool timed = false;  // time the scan launch when profiling is on
};
// vg_raycast_cells on caller-provided scratch (defined in vg_api.hip).
// dirs null: the directions are drawn on the device from `seed` (vg_philox.h).
int run_cells_in(vg_ctx *ctx, int d, int64_t n, const float *nodes, int R, const float *dirs,
                 uint64_t seed, uint32_t flags, float *t_out, int32_t *idx_out, const CellsScratch &sc,
                 const int64_t *nbr_off, const int32_t *nbr);
// Directions [n_cells][R][d] of cells first .. first + n_cells - 1 drawn from seed.
hipError_t launch_dump_dirs(int d, int64_t first, int64_t n_cells, int R, uint64_t seed, float *out,
                            hipStream_t s);

// Fixed device scratch of the allocation-free entry point (vg_noalloc.hip):
// noalloc_attach looks up its address on the current device once (called by
// vg_create); noalloc_scratch returns it (null before attach or on failure).
constexpr int64_t kNoAllocMaxRays = int64_t(1) << 22;
constexpr size_t kNoAllocCounterBytes = 256;
constexpr size_t kNoAllocBytes = kNoAllocCounterBytes + (size_t)kNoAllocMaxRays * 9 + 256;
hipError_t noalloc_attach(int device);
void *noalloc_scratch(int device);

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
  std::vector<void *> retired;  // earlier scratch blocks (a captured graph may read them)
  uint32_t *counters = nullptr;  // device [CNT_WORDS]
  int64_t last_rays = 0;
  double last_tau = 0.0;
  uint32_t *last_counters = nullptr;  // counters written by the last call (stats)
  void *batch_state = nullptr;         // graphs, tuner cache of the batched path
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> scan_events;  // pending timings
  int64_t scan_launches = 0;
  double scan_ms = 0.0;
  hipEvent_t handoff = nullptr;  // orders a new stream after the old one (vg_set_stream)
};
