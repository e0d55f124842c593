/*
 * vgraph.h -- C ABI of the MI355X (gfx950) batched RayCast library for the
 * Voronoi Graph method (Sikorski & Heida, arXiv 2405.10050).
 *
 * The library computes the RayCast of Sec. 2.2: for a ray with origin x
 * (equidistant to the known generators eta, in the cell of g = eta[0]) and
 * direction u, the first bisector hit
 *
 *     t* = min over nodes r not in eta with u.(r - g) > 0 of
 *          (|r - x|^2 - |g - x|^2) / (2 u.(r - g))          (eq. (t))
 *
 * and its argmin, optionally clipped to the unit cube [0,1]^d.  On top of it
 * sit the Monte-Carlo volume / interface-area estimators of Sec. 3.1
 * (Algorithm 3), their adjoint with respect to the generator positions, and
 * the exhaustive vertex search of Sec. 2.3 (Algorithm 2).
 *
 * Conventions shared by every call
 *  - All array arguments are DEVICE pointers on the context's device unless
 *    stated otherwise, row-major and densely packed.  The caller owns them;
 *    the library never frees or keeps them past the call.
 *  - Work is enqueued on the context's stream (vg_set_stream); calls return
 *    without synchronising unless stated otherwise.  Outputs are valid once
 *    the stream has reached the call.
 *  - Every call returns a vg_status.  Arguments are validated before any
 *    launch; on error nothing is launched and vg_last_error() describes it.
 *  - 2 <= d <= VG_MAX_DIM.  Node indices are int32 (n_nodes < 2^31).
 *  - A ray result index idx >= 0 is a node; -1 means no hit (the ray leaves
 *    to infinity); -2-(2k+s) is the face x_k = s of the unit cube (s = 0, 1).
 *  - Ties: equal t goes to the lowest node index, and a node beats a face of
 *    the cube.  The scan runs in FP32; a ray whose two best candidates are
 *    within a relative gap VG_TIE_EPS (or whose result could hinge on FP32
 *    rounding) is re-evaluated over all nodes in FP64 and flagged.
 *  - Non-finite input (NaN or Inf) is checked on the device without a
 *    synchronisation: a non-finite node coordinate makes every ray of the
 *    call, and a non-finite origin or direction makes that ray, return
 *    t = NaN, idx = -1, status VG_ST_BAD_INPUT (counted in vg_stats);
 *    Monte-Carlo sums over such rays are NaN.  vg_explore, which
 *    synchronises anyway, returns VG_EINVAL instead.  The batched calls do
 *    not check their inputs.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef VGRAPH_H
#define VGRAPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VG_MAX_DIM 16

typedef enum vg_status {
  VG_OK = 0,
  VG_EINVAL = -1,       /* bad argument (null pointer, size, dimension)      */
  VG_ENOMEM = -2,       /* device or host allocation failed                  */
  VG_EDEVICE = -3,      /* a HIP call failed                                 */
  VG_EUNSUPPORTED = -4  /* valid request outside what the library supports  */
} vg_status;

/* flags */
#define VG_CLIP (1u << 0)        /* clip rays to the unit cube                 */
#define VG_PREC_BF16X3 (1u << 1) /* Monte-Carlo scan in split BF16x3 MFMA       */
#define VG_NO_RECHECK (1u << 2)  /* skip the FP64 re-evaluation (diagnostics)  */
#define VG_INCIRCLE (1u << 3)    /* rays by the incircle RayCast of Algorithm 1
                                    with a grid index (d <= 6)                  */
#define VG_INIT_HEURISTIC (1u << 4) /* with VG_INCIRCLE on general rays: start
                                    from InitialHeuristic (|eta| >= 2)         */
#define VG_PERIODIC (1u << 5)    /* vg_explore: the periodic diagram (torus)    */
#define VG_SCAN_ORDER (1u << 6)  /* Monte-Carlo scan over the nodes sorted along
                                    a Morton curve, skipping node blocks and
                                    chunks that cannot change a ray's two best
                                    candidates (default for d <= 12 in FP32,
                                    d <= 10 in BF16x3)                         */
#define VG_INDEX_ORDER (1u << 7) /* Monte-Carlo scan over every node in index
                                    order (default above)                      */

/* per-ray status bits (uint8) */
#define VG_ST_NEAR_TIE 1  /* FP32 gap of the two best candidates below VG_TIE_EPS */
#define VG_ST_RECHECKED 2 /* result re-evaluated over all nodes in FP64          */
#define VG_ST_NO_HIT 4    /* no node ahead of the ray (t = +inf, idx = -1)       */
#define VG_ST_SUSPECT 8   /* winner nearly parallel to its bisector in FP32      */
#define VG_ST_FP64_TIE 16 /* FP64 gap below 1e-9: several answers are correct    */
#define VG_ST_BAD_INPUT 32 /* non-finite input: a node coordinate (then every ray
                              of the call), or this ray's origin or direction;
                              t = NaN, idx = -1                                 */

typedef struct vg_ctx vg_ctx;
typedef struct vg_mesh vg_mesh;

typedef struct vg_stats {
  int64_t rays;          /* rays of the last call                              */
  int64_t flagged;       /* rays re-evaluated in FP64 by the last call          */
  int64_t fp64_ties;     /* of those, rays with an FP64 near-tie                 */
  double tie_eps;        /* relative FP32 gap that triggers the FP64 recheck    */
  int64_t scan_launches; /* candidate-scan launches timed since profiling began */
  double scan_ms;        /* their summed duration (HIP events on the stream)    */
  int64_t nn_calls;      /* nearest-neighbour queries of the last VG_INCIRCLE call */
  int64_t nn_grid_calls; /* of those, queries answered by the grid (the others
                            by the cell's list of nearest nodes)             */
  int64_t bad_input_rays; /* rays of the last call answered NaN / -1 because of
                             non-finite input (VG_ST_BAD_INPUT)              */
  int64_t bad_node_values; /* non-finite node coordinates the last call saw   */
  int64_t scan_pairs;    /* ray-node pairs the last Monte-Carlo cell scan
                            evaluated on MFMA (1024 per 32x32 block; blocks
                            that provably cannot change a ray's two best
                            candidates are skipped; 0 for other calls)       */
} vg_stats;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device` with the null stream.  Allocates a
 * small amount of device memory; scratch grows on demand and is kept until
 * vg_destroy.  Returns VG_EDEVICE if the device is absent or not gfx950. */
int vg_create(int device, vg_ctx **out);
void vg_destroy(vg_ctx *ctx);
/* Bind a hipStream_t (passed as void*); NULL selects the null stream.  When
 * the stream changes, work later enqueued on the new stream waits for this
 * context's work already enqueued on the old one (an event), since calls
 * share the context's scratch and counters. */
int vg_set_stream(vg_ctx *ctx, void *hip_stream);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *vg_last_error(const vg_ctx *ctx);
/* Counters of the last raycast-type call.  Synchronises the stream. */
int vg_get_stats(vg_ctx *ctx, vg_stats *out);
/* enable != 0: record a HIP event pair around every candidate-scan kernel
 * (cell or ray scan) on the context's stream and accumulate their durations
 * into vg_stats.scan_ms / scan_launches; enable == 0 stops and clears. */
int vg_set_profiling(vg_ctx *ctx, int enable);

/* Measured peak rate of one arithmetic pipe, for reporting beside the
 * datasheet peaks: kind 0 = FP32 MFMA (v_mfma_f32_32x32x2f32), 1 = BF16 MFMA
 * (v_mfma_f32_32x32x16_bf16), 2 = FP64 vector FMA.  Runs a short
 * issue-bound kernel on every SIMD three times and returns the best rate in
 * FLOP/s (a multiply-add counts 2).  Allocates a small buffer and
 * synchronises the stream. */
int vg_peak_rate(vg_ctx *ctx, int kind, double *flops_per_s);

/* ---------------------------------------------------------------- RayCast */
/* RayCast of n_rays arbitrary rays (Sec. 2.2, eq. (t); the half-space
 * restriction is the `skip` predicate of Algorithm 1).
 *   nodes  [n_nodes][d] f32
 *   origin [n_rays][d]  f32   ray start x (equidistant to its eta)
 *   dir    [n_rays][d]  f32   direction u, used as given (not renormalised)
 *   gen    [n_rays]     i32   g = eta[0], the generator in eq. (t)
 *   excl   [n_rays][n_excl] i32, each row sorted ascending: eta (nodes never
 *          returned); may be NULL when n_excl == 0.  0 <= n_excl <= d.
 *   flags  VG_CLIP, VG_NO_RECHECK, VG_INCIRCLE, VG_INIT_HEURISTIC
 * With VG_INCIRCLE (d <= 6) each ray runs Algorithm 1 with nearest-neighbour
 * queries answered by a uniform grid over the cube (built per call), from
 * the origin or, with VG_INIT_HEURISTIC and |eta| >= 2, from
 * InitialHeuristic's point; the results are the same as the scan's (the
 * FP32 certificate and the FP64 recheck of uncertain rays), and
 * vg_stats.nn_calls counts the queries.
 * Outputs (all [n_rays]): t_out f32 (+inf when no hit), idx_out i32,
 * status_out u8 (may be NULL).  n_rays == 0 is a no-op. */
int vg_raycast(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
               int64_t n_rays, const float *origin, const float *dir,
               const int32_t *gen, const int32_t *excl, int n_excl,
               uint32_t flags, float *t_out, int32_t *idx_out,
               uint8_t *status_out);

/* vg_raycast with FP64 origins and directions (a vertex and a
 * SearchDirection of Algorithm 2 are FP64): origin, dir [n_rays][d] f64.
 * The scan runs on their FP32 rounding with the error of that rounding in
 * its certificate, and the recheck and the winner's t* use the FP64 values
 * (the exhaustive search casts its edge rays this way).  flags VG_CLIP,
 * VG_INCIRCLE, VG_INIT_HEURISTIC; status_out may be NULL.  Reads the
 * recheck queue's length back: synchronises the stream. */
int vg_raycast_f64(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                   int64_t n_rays, const double *origin, const double *dir,
                   const int32_t *gen, const int32_t *excl, int n_excl,
                   uint32_t flags, float *t_out, int32_t *idx_out,
                   uint8_t *status_out);

/* Monte-Carlo rays of every cell (Algorithm 3): ray k of cell i starts at
 * x_i with eta = {i} and direction dirs[i][k], clipped to the unit cube
 * (VG_CLIP is implied).  The candidate scan is the dense contraction of the
 * directions with the nodes inverted about x_i, on MFMA.  With VG_INCIRCLE
 * the rays are cast instead by the incircle iteration of Algorithm 1, its
 * nearest-neighbour queries answered by a uniform grid over the cube (built
 * per call; nodes must lie in [0,1]^d; d <= 6, FP32 only) or, when it
 * provably holds every node that matters, by the cell's list of nearest
 * nodes, which also gives the first candidate; results are the same (the
 * certificate and the FP64 recheck are shared), and vg_stats.nn_calls and
 * nn_grid_calls count the queries.
 * Node order of the dense scan: with VG_SCAN_ORDER (the default for
 * d <= 12 in FP32 and d <= 10 in BF16x3) the call first sorts a copy of the
 * nodes along a Morton curve of all their coordinates, scaled to the cloud's
 * bounding box (a pass of plain kernels, O(n log^2 n)); each cell then scans
 * from its own place in that order outwards and skips a 32-node block, or a
 * whole chunk of nodes, when a rigorous bound on u.r~ over it is below
 * every ray's current second-best value.  The bounds need unit directions
 * (up to rounding): a workgroup that holds a longer one skips nothing.  The
 * skip is exact: every output equals the one of the scan over all nodes in
 * index order (VG_INDEX_ORDER, the default above those dimensions, where
 * uniform clouds leave little to skip); vg_stats.scan_pairs counts the
 * ray-node pairs evaluated.
 * Neighbour-restricted scans (vg_mc_volume_area_nbr) keep their list order.
 *   dirs [n_nodes][rays_per_cell][d] f32 unit vectors
 *   flags VG_PREC_BF16X3, VG_NO_RECHECK, VG_INCIRCLE, VG_SCAN_ORDER,
 *         VG_INDEX_ORDER (not both)
 * Outputs [n_nodes * rays_per_cell], cell-major: t_out, idx_out, status_out
 * (may be NULL).  1 <= rays_per_cell <= 4096. */
int vg_raycast_cells(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                     int rays_per_cell, const float *dirs, uint32_t flags,
                     float *t_out, int32_t *idx_out, uint8_t *status_out);

/* vg_raycast_cells with the directions drawn on the device instead of read
 * from memory (Sec. 3.1: u uniform on the unit sphere, the normalised
 * standard normal vector drawn in Algorithm 3).  Direction of ray k of cell
 * i, component c: Philox4x32-10 (Salmon et al., SC'11) with counter
 * (c / 4, k, i mod 2^32, i / 2^32) and key (seed mod 2^32, seed / 2^32)
 * gives words w0..w3; pair p = (c mod 4) / 2 takes a = w[2p], b = w[2p+1];
 * u1 = (a + 1/2) 2^-32, u2 = b 2^-32, rho = sqrt(-2 ln u1), theta = 2 pi u2
 * (Box-Muller, FP64); z_c = rho cos theta (c even) or rho sin theta (c odd);
 * u_c = fp32(z_c / sqrt(z_0^2 + z_1^2 + ...)), the squares summed in order
 * without fused multiply-add.  The directions are never stored: every
 * kernel that needs one recomputes it, and vg_dump_dirs writes them out.
 * Same flags and outputs as vg_raycast_cells (VG_INCIRCLE is
 * VG_EUNSUPPORTED). */
int vg_raycast_cells_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                            int rays_per_cell, uint64_t seed, uint32_t flags,
                            float *t_out, int32_t *idx_out, uint8_t *status_out);

/* The directions that the seeded calls draw for cells first_cell ..
 * first_cell + n_cells - 1: out [n_cells][rays_per_cell][d] f32 (DEVICE).
 * The same function of (seed, cell, ray) as in the kernels, bit for bit. */
int vg_dump_dirs(vg_ctx *ctx, int d, int64_t first_cell, int64_t n_cells, int rays_per_cell,
                 uint64_t seed, float *out);

/* vg_raycast_cells for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the recheck queue, the
 * status bytes (when status_out is NULL) and the counters in a fixed scratch
 * array of the library (about 36 MiB per device, held from library load
 * until the process ends).  No call allocates or frees device memory.
 * n_nodes * rays_per_cell <= VG_NOALLOC_MAX_RAYS, else VG_EINVAL; VG_INCIRCLE
 * and VG_SCAN_ORDER are VG_EUNSUPPORTED (the scan runs in index order, with
 * the same outputs); other arguments, flags and outputs as
 * vg_raycast_cells.  Every call on one device shares that array and the
 * array keeps the last call's contents (each call clears its counters
 * first): calls that overlap on one device (other streams, other contexts
 * or threads) race and give wrong results.  vg_get_stats reads the array's
 * counters of the last call. */
#define VG_NOALLOC_MAX_RAYS (1ll << 22)
int vg_raycast_cells_noalloc(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                             int rays_per_cell, const float *dirs, uint32_t flags,
                             float *t_out, int32_t *idx_out, uint8_t *status_out);

/* ------------------------------------------------ Monte-Carlo estimators */
/* Sec. 3.1 / Algorithm 3 with f = 1: for every cell i, with l = t* of its
 * rays and S = S_{d-1} = 2 pi^{d/2} / Gamma(d/2),
 *   volume[i]  = S/(d n)     sum_k l_k^d
 *   energy2[i] = S/((d+2) n) sum_k l_k^{d+2}   (= int_{C_i} |y - x_i|^2 dy)
 *   area(i,j)  = S/n sum_{k: j_k = j} l_k^{d-1} / |n_ij . u_k|   (eq. dS-dA)
 * where n = rays_per_cell and n_ij is the unit normal of the facet (for a
 * node j, (x_j - x_i)/|x_j - x_i|; for a cube face, e_k).  Facets of cell i
 * are written to row i of facet_j / facet_area, sorted by j as signed int32
 * (cube faces, negative codes, first), facet_count[i] entries; the rest of
 * the row is left untouched.
 *   t_out, idx_out [n_nodes*n] (required: the adjoint reads them back),
 *   status_out [n_nodes*n] u8 or NULL,
 *   volume [n_nodes] f32 (required), energy2 [n_nodes] f32 or NULL,
 *   facet_j [n_nodes][n] i32, facet_area [n_nodes][n] f32,
 *   facet_count [n_nodes] i32 -- all three NULL to skip the facets. */
int vg_mc_volume_area(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                      int rays_per_cell, const float *dirs, uint32_t flags,
                      float *t_out, int32_t *idx_out, uint8_t *status_out,
                      float *volume, float *energy2, int32_t *facet_j,
                      float *facet_area, int32_t *facet_count);

/* vg_mc_volume_area with the directions drawn on the device from `seed`, as
 * in vg_raycast_cells_seeded (no dirs array anywhere). */
int vg_mc_volume_area_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                             int rays_per_cell, uint64_t seed, uint32_t flags,
                             float *t_out, int32_t *idx_out, uint8_t *status_out,
                             float *volume, float *energy2, int32_t *facet_j,
                             float *facet_area, int32_t *facet_count);

/* vg_mc_volume_area with each cell's candidate scan restricted to a list of
 * its neighbours: once the Voronoi diagram is known, a ray of cell i can only
 * leave through a facet shared with a neighbouring cell (the remark closing
 * Sec. 3.1), so t* over the list equals t* over all nodes whenever the list
 * of every cell holds all generators whose cells share a facet with it (a
 * superset is fine; vg_tuple_neighbors builds it from vg_explore's vertices).
 * Rays the FP32 certificate cannot settle are re-evaluated over ALL nodes in
 * FP64, as in vg_mc_volume_area.  Same flags and outputs.
 *   nbr_offsets [n_nodes+1] i64, nondecreasing, nbr_offsets[0] = 0;
 *   nbr [nbr_offsets[n_nodes]] i32: row i lists cell i's candidates (any
 *   order, without i).  Entries outside [0, n_nodes) are ignored; a missing
 *   neighbour gives wrong t* for the rays that leave through its facet. */
int vg_mc_volume_area_nbr(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                          const int64_t *nbr_offsets, const int32_t *nbr,
                          int rays_per_cell, const float *dirs, uint32_t flags,
                          float *t_out, int32_t *idx_out, uint8_t *status_out,
                          float *volume, float *energy2, int32_t *facet_j,
                          float *facet_area, int32_t *facet_count);

/* Generator adjacency of a set of Voronoi vertices (Sec. 2.1: a vertex is
 * equidistant to its d+1 generators), as CSR: j is listed in row i when some
 * tuple holds both i and j.  For the vertex set of vg_explore these are the
 * neighbouring cells of each generator.
 *   sigma [n_tuples][d+1] i32 (DEVICE; entries in [0, n_nodes), else
 *         VG_EINVAL);
 *   offsets [n_nodes+1] i64 and nbr [nbr_capacity] i32 (DEVICE outputs, both
 *         NULL to count only); rows sorted ascending, no duplicates;
 *   *nnz (HOST) receives the number of entries; nbr_capacity < *nnz is
 *         VG_EINVAL (n_tuples*(d+1)*d always suffices).
 * At most 2^31 - 1 ordered tuple pairs (VG_EUNSUPPORTED beyond).  Allocates
 * temporary device memory and synchronises the stream. */
int vg_tuple_neighbors(vg_ctx *ctx, int d, int64_t n_nodes, int64_t n_tuples,
                       const int32_t *sigma, int64_t *offsets, int32_t *nbr,
                       int64_t nbr_capacity, int64_t *nnz);

/* Integrals of a function f over the cells and their facets, following
 * Algorithm 3 (Sec. 3.1) with its inner loop of m draws per ray.  Two calls,
 * with the caller evaluating f in between:
 *
 * vg_mc_sample_points writes, for every ray k of cell i (l = t*, from
 * vg_mc_volume_area or vg_mc_volume_area_nbr with the same dirs), the hit
 * point x_i + l u followed by the interior points x_i + t_s l u:
 *   t [n_nodes*n] f32, tsamp [n_nodes][n][m] f32 in (0, 1) (the draws; may be
 *   NULL when m == 0), points [n_nodes][n][m+1][d] f32 (output).
 *
 * vg_mc_integrals takes fvals [n_nodes][n][m+1] f32 = f at those points and
 * writes, with S = S_{d-1},
 *   fint_volume[i] = S/(n m) sum_k sum_s f(x_i + t_ks l_k u_k) t_ks^{d-1} l_k^d
 *   F(i, j)        = S/n sum_{k: j_k = j} f(x_i + l_k u_k) l_k^{d-1} / |n_ij . u_k|
 * The normalisation S/(n m) is Algorithm 3's (the volume element in polar
 * coordinates is t^{d-1} l^d dt dS).  F(i, j) goes to fint_facet [n_nodes][n]
 * in the row layout of vg_mc_volume_area: facet_j / facet_count are written
 * too, with the same values.  fint_volume may be NULL when m == 0; the three
 * facet arrays are all set or all NULL.  0 <= m <= 1024. */
int vg_mc_sample_points(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                        int rays_per_cell, const float *dirs, const float *t, int m,
                        const float *tsamp, float *points);
int vg_mc_integrals(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                    int rays_per_cell, const float *t, const int32_t *idx, int m,
                    const float *tsamp, const float *fvals, float *fint_volume,
                    int32_t *facet_j, float *fint_facet, int32_t *facet_count);

/* Adjoint of vg_mc_volume_area with the directions frozen: writes
 *   grad_nodes[n_nodes][d] = d/dX ( sum_i g_volume[i] volume[i]
 *        + g_energy2[i] energy2[i] + sum_{i,f} g_facet_area[i][f] area(i,f) )
 * using the closed-form derivative of t* through the winning bisector
 * (t = |x_j - x_i|^2 / (2 u.(x_j - x_i)) for a node, (s - x_ik)/u_k for a
 * cube face).  t, idx, facet_j, facet_count are the forward outputs.
 * g_volume, g_energy2 [n_nodes] and g_facet_area [n_nodes][n] may each be
 * NULL (zero).  Deterministic: the scatter onto the winning generators uses
 * per-node fixed-point integer accumulation.  grad_nodes is overwritten. */
int vg_mc_backward(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                   int rays_per_cell, const float *dirs, const float *t,
                   const int32_t *idx, const int32_t *facet_j,
                   const int32_t *facet_count, const float *g_volume,
                   const float *g_energy2, const float *g_facet_area,
                   float *grad_nodes);

/* vg_mc_backward of a seeded forward call (directions drawn from `seed`). */
int vg_mc_backward_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                          int rays_per_cell, uint64_t seed, const float *t,
                          const int32_t *idx, const int32_t *facet_j,
                          const int32_t *facet_count, const float *g_volume,
                          const float *g_energy2, const float *g_facet_area,
                          float *grad_nodes);

/* ------------------------------------------------------ uneven batches */
/* One independent RayCast problem of vg_raycast_batched: the arguments of
 * vg_raycast (same layouts and meanings; status_out may be NULL, excl may be
 * NULL when n_excl == 0). */
typedef struct vg_rays_problem {
  int d;                /* 2..VG_MAX_DIM                                */
  int n_excl;           /* 0..d                                         */
  int64_t n_nodes;      /* >= 1                                         */
  const float *nodes;   /* [n_nodes][d]                                 */
  int64_t n_rays;       /* >= 0                                         */
  const float *origin;  /* [n_rays][d]                                  */
  const float *dir;     /* [n_rays][d]                                  */
  const int32_t *gen;   /* [n_rays]                                     */
  const int32_t *excl;  /* [n_rays][n_excl], rows sorted ascending      */
  float *t_out;         /* [n_rays]                                     */
  int32_t *idx_out;     /* [n_rays]                                     */
  uint8_t *status_out;  /* [n_rays] or NULL                             */
} vg_rays_problem;

/* vg_raycast (Sec. 2.2, eq. (t); the half-space restriction of Algorithm 1)
 * over many independent problems of different d, node set and ray count in
 * one persistent scan launch: workgroups take (problem, 256-ray tile) items
 * from a device counter, largest problems first; then one FP64 re-evaluation
 * pass over the flagged rays of every problem.  Each ray's result equals
 * what vg_raycast returns for it.  flags: VG_CLIP (applies to every problem);
 * VG_NO_RECHECK is not supported here (VG_EUNSUPPORTED).  The table `probs`
 * is a HOST array read during the call only; the launches are captured into
 * a hipGraph per distinct table and replayed when the same table recurs. */
int vg_raycast_batched(vg_ctx *ctx, int n_problems, const vg_rays_problem *probs,
                       uint32_t flags);

/* One independent point cloud of an uneven batch of Monte-Carlo raycasts. */
typedef struct vg_cells_problem {
  int d;                /* 2..VG_MAX_DIM                                */
  int rays_per_cell;    /* 1..4096                                      */
  int64_t n_nodes;      /* >= 1                                         */
  const float *nodes;   /* [n_nodes][d]                                 */
  const float *dirs;    /* [n_nodes][rays_per_cell][d]                  */
  float *t_out;         /* [n_nodes * rays_per_cell]                    */
  int32_t *idx_out;     /* [n_nodes * rays_per_cell]                    */
  uint8_t *status_out;  /* [n_nodes * rays_per_cell] or NULL            */
} vg_cells_problem;

/* vg_raycast_cells (the Monte-Carlo rays of Algorithm 3) over many clouds of
 * different d, N and rays_per_cell in one graph launch: one launch of the
 * single-cloud scan per cloud (the exact-K kernel of its d, in the tile shape
 * tuned for its bucket), largest clouds first, spread over four parallel
 * graph branches so the clouds' launch tails overlap; then one FP64 recheck
 * of the flagged rays of every cloud.  Each ray's result equals what
 * vg_raycast_cells returns for it.
 * flags: VG_PREC_BF16X3; VG_NO_RECHECK is VG_EUNSUPPORTED.  The problem table
 * is a HOST array read during the call only; the launches are captured into
 * a hipGraph per distinct table and replayed when the same table recurs (at
 * most 8 graphs are kept per context).  With every status_out set, a tuner
 * times half, the default and twice the default rays per workgroup on a probe
 * of each (ceil(d/2), log2 N, rays_per_cell, precision) bucket on first sight
 * (timings cached in $VG_TUNE_CACHE, default $HOME/.cache/vgraph_tune.txt)
 * and each cloud uses its bucket's fastest.  Errors: VG_EINVAL for a bad
 * table entry (d outside [2, 16] is VG_EUNSUPPORTED), VG_ENOMEM when the
 * queue or table cannot be allocated. */
int vg_raycast_cells_batched(vg_ctx *ctx, int n_problems,
                             const vg_cells_problem *probs, uint32_t flags);

/* Heuristic Monte-Carlo integrals (Sec. 3.3) over the diagram clipped to the
 * unit cube, from its vertex set (vg_explore with VG_CLIP: sigma, coords)
 * and the Monte-Carlo facet rows of every cell (vg_mc_volume_area: facet_j,
 * facet_area, facet_count; a face is -2-(2k+s) there and n_nodes + 2k + s in
 * sigma).  For facet (i, j): V_ij = the vertices whose key holds i and j
 * (K_ij), y_ij = their mean, F_ij = A_ij (d/(d+1) mean f(V_ij) + 1/(d+1)
 * f(y_ij)); the cell integral sums the pyramid rule of eq. (leibniz-int)
 * over the facets with apex x_i: sum_j h_ij/d (d/(d+1) F_ij + 1/(d+1) A_ij
 * f(x_i)), and the volume is sum_j h_ij A_ij / d, with h_ij = |x_j - x_i|/2
 * or the distance of x_i to the face.  Two calls, the caller evaluating f in
 * between:
 *
 * vg_hmc_centroids: centroid [n_nodes][rays_per_cell][d] f32 and kcount
 *   [n_nodes][rays_per_cell] i32 (K_ij) of every facet row.
 * vg_hmc_integrals: with f at the vertices f_vertex [V] f32, at the
 *   centroids f_centroid [n_nodes][rays_per_cell] f32 and at the generators
 *   f_node [n_nodes] f32: fint_facet [n_nodes][rays_per_cell] f32 (F_ij,
 *   aligned with the facet rows), fint_cell [n_nodes] f32, volume
 *   [n_nodes] f32.
 * All arrays are DEVICE, sigma [V][d+1] i32, coords [V][d] f64.  Rows past
 * facet_count are not touched.  A facet row whose pair no vertex holds, or
 * out-of-range keys or codes, give VG_EINVAL.  Both calls allocate
 * temporary device memory (the cells' vertex lists, one sort) and
 * synchronise the stream; results are bitwise reproducible. */
int vg_hmc_centroids(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_vertices,
                     const int32_t *sigma, const double *coords, int rays_per_cell,
                     const int32_t *facet_j, const int32_t *facet_count, float *centroid,
                     int32_t *kcount);
int vg_hmc_integrals(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_vertices,
                     const int32_t *sigma, const float *f_vertex, int rays_per_cell,
                     const int32_t *facet_j, const float *facet_area, const int32_t *facet_count,
                     const float *f_centroid, const float *f_node, float *fint_facet,
                     float *fint_cell, float *volume);

/* ------------------------------------------------------ exhaustive search */
/* Algorithm 2 (VoronoiGraph) on the unbounded diagram: every Voronoi vertex
 * keyed by its sorted (d+1)-tuple of generators, with FP64 coordinates
 * solved from the tuple, and every unbounded edge as (vertex, omitted
 * generator).  Rays are cast without clipping, in batches of one
 * breadth-first level; the edge visit counts and the vertex set live in
 * device hash tables.  `descent_draws` is a HOST array [n_draws][d] f64 of
 * standard normal draws consumed in order by Descent.
 * flags: 0, or VG_CLIP for the diagram clipped to the unit cube [0,1]^d (the
 * cells C_i intersected with the cube).  Its vertices are fixed by d+1
 * constraints, generators and cube faces: a key holds the generator indices,
 * then n_nodes + 2k + s for each face x_k = s the vertex lies on.  The search
 * starts at the corner 0 (no Descent: draws may be NULL), rays are clipped,
 * and there are no unbounded edges.  n_nodes >= 1 then.
 * VG_INCIRCLE (d <= 6), optionally with VG_INIT_HEURISTIC, casts the edge
 * rays by Algorithm 1 (as vg_raycast); vg_mesh_num_nn_calls then counts its
 * nearest-neighbour queries (the measure of Table nncalls).
 * VG_PERIODIC (d <= 8; excludes VG_CLIP and VG_INCIRCLE) searches the
 * periodic diagram, the torus R^d / Z^d of the periodic boundary conditions
 * behind Table empscaling, for nodes in [0,1)^d (VG_EINVAL otherwise).  A
 * key entry is a node image x_i + k, coded i*3^d + sum_a (k_a + 1) 3^a with
 * k in {-1,0,1}^d; each key is sorted and translated by a lattice vector so
 * that its first node has k = 0, and coords are solved in that frame from
 * the exact images.  Rays run over the images inside [-w, 1+w]^d (FP32
 * rows; the FP64 recheck reads the exact images), and every new vertex's
 * ball is checked to lie inside that layer; otherwise the search restarts
 * with w doubled, up to w = 1.  Needs n_nodes * 3^d < 2^31 - 1 and every
 * vertex ball radius below 1/2 (VG_EUNSUPPORTED otherwise, e.g. for a
 * handful of nodes).  There are no unbounded edges.
 * Synchronises the stream.  The result is library-owned: query it, copy it
 * out, free it. */
int vg_explore(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
               const double *descent_draws, int n_draws, uint32_t flags,
               vg_mesh **out);
int64_t vg_mesh_num_vertices(const vg_mesh *mesh);
int64_t vg_mesh_num_unbounded(const vg_mesh *mesh);
int64_t vg_mesh_num_raycasts(const vg_mesh *mesh);
int64_t vg_mesh_num_nn_calls(const vg_mesh *mesh);
/* HOST outputs: sigma [V][d+1] (tuples in discovery order), coords [V][d] f64
 * or NULL, b_sigma [B][d+1] or NULL, b_omit [B] or NULL. */
int vg_mesh_copy(const vg_mesh *mesh, int32_t *sigma, double *coords,
                 int32_t *b_sigma, int32_t *b_omit);
void vg_mesh_free(vg_mesh *mesh);

#ifdef __cplusplus
}
#endif
#endif /* VGRAPH_H */
