// The incircle RayCast of Algorithm 1 on the GPU, with a uniform-grid
// nearest-neighbour index: for the Monte-Carlo rays of every cell (eta =
// {i}, origin x_i, clipped to the unit cube) and for general rays (an origin
// equidistant to eta, e.g. the exhaustive search's edge rays).  A sublinear
// alternative to the dense scan when N is large and d small.
//
// Index: G^d cells over [0,1]^d (about two nodes per cell), nodes sorted by
// cell (counting sort), their coordinates stored in cell order.  A node
// outside [0,1]^d would escape the ring bound below, so its presence sends
// every ray to the FP64 recheck.
//
// nn(q): the nearest node to q whose `skip` predicate of Algorithm 1 is false
// (u.(x_k - x_g) > 0: the half-space ahead of the ray; eta excluded), with
// the second nearest.  Distances are taken from coordinates relative to the
// ray's generator x_g, so their rounding scales with the cell rather than
// with the cube.  Cells are visited in Chebyshev rings around q's (clamped)
// cell; a node outside ring rho - 1 is at least (rho - 1) h away in one
// coordinate and at least q's distance to the cube in the others, so the
// search stops once that bound exceeds every distance that could still
// change the answer or its certificate.  A query that would visit more than
// a budget of ring offsets gives up, and its ray goes to the FP64 recheck.
//
// Monte-Carlo rays: Algorithm 1 needs a first generator candidate, and its
// InitialHeuristic is undefined for |eta| = 1.  Any eligible node k gives an
// upper bound t_k = |x_k - x_i|^2 / (2 u.(x_k - x_i)) on the result (eq. (t)
// with r = x_i), so the first candidate is the best of the cell's K nearest
// nodes (one search per cell, shared by its R rays): usually the winner
// itself, so one nn call confirms it.  From there the loop of Algorithm 1
// runs: candidate r' = x_i + t u, j = nn(r'); j = k ends it.  When no listed
// node crosses the ray before the cube, the ray's exit point is tested
// instead: if no eligible node is nearer to it than x_i, the exit point lies
// in cell i and the cube face is the result; otherwise the loop starts from
// the node nn returned.  Every candidate has t below the exit, so it lies
// inside the cube, where the grid query is cheap.  The cell's list answers a
// query by itself when it provably holds every node that matters.
//
// Two passes for the Monte-Carlo rays: one thread per ray casts it while the
// cell's list answers its queries (almost always); the few rays that need
// the grid are queued and resumed by a second pass, so that grid walks do
// not hold up whole waves.
//
// General rays: Algorithm 1 as printed, from the origin or from
// InitialHeuristic's point (incircle_ray below).
//
// Certificate: at the final candidate, the gap between the squared distances
// of the nearest and second-nearest eligible node (the face test: between
// the nearest eligible node and x_i) equals 2 u.(x_k - x_g)(t_k - t*) for the
// runner-up k, so a gap above the FP32 error of the distances certifies the
// result.  Other rays (and iteration caps, nearly grazing winners, queries
// that gave up) are queued for the FP64 recheck over all nodes.
#include <hipcub/hipcub.hpp>

#include "vg_dfloat.h"
#include "vg_internal.h"

namespace vg {
namespace {

constexpr int NT = 256;
constexpr int kMaxIter = 64;
// Ring offsets one query may visit.  A query point far outside the cube sees
// a whole face nearly equidistant, and a ray with no eligible node sweeps
// the grid: past the budget the query gives up (i1 = kGaveUp) and the ray
// goes to the FP64 recheck over all nodes.  Where a full sweep costs at most
// kFullSweep offsets (every grid of N = 1000 nodes in d = 2..5) the budget
// is that sweep, so no query gives up; on larger grids it is kRingBudget,
// about twelve times a local query in 3-D, for the Monte-Carlo rays, and
// kRayRingBudget for general rays: a breadth-first level of the search waits
// for its slowest ray, and the rays near the hull of the unbounded diagram,
// which find no eligible node, would each walk the whole budget; the FP64
// recheck settles them faster.
constexpr int kFullSweep = 1 << 15;
constexpr int kRingBudget = 1 << 12;
constexpr int kRayRingBudget = 1 << 9;
// Lanes sharing one ray's grid queries where rays are few for the GPU (a
// breadth-first level of the search, the rays the lists could not answer):
// each query walks grid cells with dependent loads, and eight lanes split
// its rings.
constexpr int kRayLanes = 8;
constexpr int32_t kGaveUp = -2;

// Cell of every node; a node outside [0,1]^d (clamped into a boundary cell,
// where the ring bound does not hold for it) sets *outside.
__global__ void grid_count_kernel(const float *__restrict__ X, int64_t n, int d, int G,
                                  int32_t *__restrict__ cell_of, uint32_t *__restrict__ counts,
                                  uint32_t *__restrict__ outside) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  int64_t c = 0;
  for (int k = 0; k < d; ++k) {
    const float x = X[i * d + k];
    if (!(x >= 0.f && x <= 1.f)) atomicOr(outside, 1u);
    int q = (int)floorf(x * (float)G);
    q = q < 0 ? 0 : (q >= G ? G - 1 : q);
    c = c * G + q;
  }
  cell_of[i] = (int32_t)c;
  atomicAdd(&counts[c + 1], 1u);
}

// Scatter every node into its cell's range (order within a cell is
// arbitrary; the nearest-neighbour query breaks distance ties by index).
__global__ void grid_fill_kernel(const float *__restrict__ X, int64_t n, int d, const int32_t *__restrict__ cell_of,
                                 const uint32_t *__restrict__ start, uint32_t *__restrict__ cursor,
                                 float *__restrict__ Xs, int32_t *__restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int32_t c = cell_of[i];
  const uint32_t p = start[c] + atomicAdd(&cursor[c], 1u);
  ids[p] = (int32_t)i;
  for (int k = 0; k < d; ++k) Xs[(int64_t)p * d + k] = X[i * d + k];
}

// Error bound of a difference da - db of squared distances from a computed
// candidate q = x_i + t u to two nodes a, b, each distance evaluated from
// coordinates relative to x_i, e = t u - (x_a - x_i):
//  - evaluation: coordinate k of e carries at most (|t u_k| + |x_ak - x_ik|
//    + |e_k|) 2^-24, a vector of norm at most 2 (t + s_a) 2^-24 (s_a =
//    sqrt(da), |x_a - x_i| <= t + s_a), which moves da by 2 s_a times that;
//    the sum of squares adds (d + 1) 2^-24 da;
//  - position: q lies within `shift` of the exact candidate, which moves
//    da - db by at most 2 shift (s_a + s_b).
// Times 4 for safety.  All terms scale with the cell, not with the cube.
__device__ __forceinline__ float gap_tol(float da, float db, float shift, float t, int d) {
  const float sa = sqrtf(da), sb = sqrtf(db);
  const float eval = (4.f * (sa * (t + sa) + sb * (t + sb)) + (float)(d + 1) * (da + db)) * 0x1p-24f;
  return 4.f * (eval + 2.f * shift * (sa + sb));
}

// Slack of the ring bound for the rounding of cell indices (of q and of the
// nodes) and of q's absolute coordinates.
constexpr float kRingSlack = 0x1p-20f;

struct GridView {
  const float *X;         // [n][d] nodes in cell order
  const int32_t *id;      // [n] node index of each sorted slot
  const uint32_t *start;  // [G^d + 1]
  int G;
  float h;
  const uint32_t *outside;  // nonzero: some node lies outside [0,1]^d, and
                            // every query defers to the FP64 recheck
  int budget;               // ring offsets one query may visit
};

// Top-2 nearest eligible nodes (squared distances) of the query point
// q = x_g + qr, from coordinates relative to the ray's generator x_g (|qr| =
// T); eligible means u.(x_k - x_g) > 0 (the skip predicate of Algorithm 1)
// and k not in ex[0 .. n_ex) (eta).  A node whose squared distance exceeds
// ref + gap_tol(ref, .) with ref = min(d1, limit) cannot change the caller's
// decision or its certificate, so the ring search stops once every
// unvisited node is that far (or beyond d2).  A node outside ring rho - 1 of
// q's (clamped) cell is at least (rho - 1) h away in one coordinate and at
// least q's distance to the cube in the others, so the bound adds that
// distance when q lies outside.  `shift` bounds the distance of q from the
// exact point (for gap_tol).
// The eligible nodes of one grid cell into the running nearest two (d1 with
// node i1, d2); equal distances go to the lower node index.
template <int DK>
__device__ __forceinline__ void scan_cell(const GridView &g, int64_t cell, int d, const float (&xg)[DK],
                                          const float (&qr)[DK], const float (&u)[DK], const int32_t *ex, int n_ex,
                                          int32_t &i1, float &d1, float &d2) {
  for (uint32_t p = g.start[cell]; p < g.start[cell + 1]; ++p) {
    const int32_t node = g.id[p];
    bool in_eta = false;
    for (int e = 0; e < n_ex; ++e) in_eta |= ex[e] == node;
    if (in_eta) continue;
    const float *xp = g.X + (int64_t)p * d;
    float den = 0.f, dist = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {
        const float ek = xp[k] - xg[k];
        den = __builtin_fmaf(u[k], ek, den);
        const float e = qr[k] - ek;
        dist = __builtin_fmaf(e, e, dist);
      }
    }
    if (!(den > 0.f)) continue;  // skip: not ahead of the ray
    if (dist < d1 || (dist == d1 && node < i1)) {
      d2 = d1;
      d1 = dist;
      i1 = node;
    } else if (dist < d2) {
      d2 = dist;
    }
  }
}

// Query cell of q and its squared distance to the cube (0 inside).
template <int DK>
__device__ __forceinline__ float query_cell(const GridView &g, int d, const float (&xg)[DK], const float (&qr)[DK],
                                            int (&c)[DK]) {
  float out2 = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    const float qa = xg[k] + qr[k];
    int v = k < d ? (int)floorf(qa * (float)g.G) : 0;
    c[k] = v < 0 ? 0 : (v >= g.G ? g.G - 1 : v);
    const float o = k < d ? fmaxf(0.f, fmaxf(-qa, qa - 1.f)) : 0.f;
    out2 = __builtin_fmaf(o, o, out2);
  }
  return out2 * (1.f - 0x1p-20f);
}

template <int DK>
__device__ void nn2(const GridView &g, int d, const float (&xg)[DK], const float (&qr)[DK], const float (&u)[DK],
                    float T, const int32_t *ex, int n_ex, float limit, float shift, int32_t &i1, float &d1,
                    float &d2) {
  int c[DK];
  const float out2 = query_cell<DK>(g, d, xg, qr, c);
  i1 = -1;
  d1 = d2 = __builtin_inff();
  int budget = g.budget;
  for (int rho = 0; rho < g.G; ++rho) {
    if (rho >= 1) {
      const float lb = fmaxf(0.f, (float)(rho - 1) * g.h - kRingSlack);
      const float lb2 = lb * lb + out2;
      const float ref = fminf(d1, limit);
      if (lb2 > d2 || lb2 > ref + gap_tol(ref, lb2, shift, T, d)) break;
    }
    // offsets o in [-rho, rho]^d with max |o_k| = rho, as a mixed-radix counter
    const int span = 2 * rho + 1;
    int o[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) o[k] = -rho;
    for (;;) {
      if (--budget < 0) {
        i1 = kGaveUp;
        return;
      }
      bool on_ring = false, inside = true;
      int64_t cell = 0;
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        if (k < d) {
          const int ck = c[k] + o[k];
          on_ring |= (o[k] == rho || o[k] == -rho);
          inside &= (ck >= 0 && ck < g.G);
          cell = cell * g.G + ck;
        }
      }
      if (on_ring && inside) scan_cell<DK>(g, cell, d, xg, qr, u, ex, n_ex, i1, d1, d2);
      // next offset
      int k = d - 1;
      while (k >= 0) {
        if (++o[k] <= rho) break;
        o[k] = -rho;
        --k;
      }
      if (k < 0 || span == 1) break;
    }
  }
}

// nn2 by a group of GL lanes of one wave (aligned, GL dividing 64), all in
// the same call with the same arguments: the lanes stride over the offsets
// of each ring, each keeping the nearest two of its own cells, and after
// every ring their states are merged by shuffles within the group, so every
// lane holds the same (i1, d1, d2).  The nearest node (lowest
// index on equal distances) and the second distance do not depend on the
// order in which cells are visited, and a ring is skipped as a whole when it
// would overrun the budget (the serial walk gives up inside that ring), so
// the result is nn2's.
template <int DK, int GL>
__device__ void nn2_group(const GridView &g, int d, const float (&xg)[DK], const float (&qr)[DK],
                          const float (&u)[DK], float T, const int32_t *ex, int n_ex, float limit, float shift,
                          int lane, int32_t &i1, float &d1, float &d2) {
  int c[DK];
  const float out2 = query_cell<DK>(g, d, xg, qr, c);
  // each lane's own nearest two over the cells it visited (disjoint across
  // the group); (i1, d1, d2) is their merge after every ring
  int32_t li1 = -1;
  float ld1 = __builtin_inff(), ld2 = __builtin_inff();
  i1 = -1;
  d1 = d2 = __builtin_inff();
  int budget = g.budget;
  for (int rho = 0; rho < g.G; ++rho) {
    if (rho >= 1) {
      const float lb = fmaxf(0.f, (float)(rho - 1) * g.h - kRingSlack);
      const float lb2 = lb * lb + out2;
      const float ref = fminf(d1, limit);
      if (lb2 > d2 || lb2 > ref + gap_tol(ref, lb2, shift, T, d)) break;
    }
    const int span = 2 * rho + 1;
    int count = 1;
    for (int k = 0; k < d; ++k) count *= span;
    budget -= count;
    if (budget < 0) {
      i1 = kGaveUp;
      return;
    }
    for (int idx = lane; idx < count; idx += GL) {
      bool on_ring = false, inside = true;
      int64_t cell = 0;
      int rem = idx;
      int o[DK];
#pragma unroll
      for (int k = DK - 1; k >= 0; --k) {
        if (k < d) {
          o[k] = rem % span - rho;
          rem /= span;
        } else {
          o[k] = 0;
        }
      }
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        if (k < d) {
          const int ck = c[k] + o[k];
          on_ring |= (o[k] == rho || o[k] == -rho);
          inside &= (ck >= 0 && ck < g.G);
          cell = cell * g.G + ck;
        }
      }
      if (on_ring && inside) scan_cell<DK>(g, cell, d, xg, qr, u, ex, n_ex, li1, ld1, ld2);
    }
    i1 = li1;
    d1 = ld1;
    d2 = ld2;
#pragma unroll
    for (int off = 1; off < GL; off <<= 1) {
      const float od1 = __shfl_xor(d1, off);
      const int32_t oi1 = __shfl_xor(i1, off);
      const float od2 = __shfl_xor(d2, off);
      const float nd2 = fminf(fminf(d2, od2), fmaxf(d1, od1));
      if (od1 < d1 || (od1 == d1 && oi1 >= 0 && (i1 < 0 || oi1 < i1))) {
        d1 = od1;
        i1 = oi1;
      }
      d2 = nd2;
    }
  }
}

// nn2 by one lane (GL = 1) or by a group of GL lanes.
template <int DK, int GL>
__device__ __forceinline__ void nn2_lanes(const GridView &g, int d, const float (&xg)[DK], const float (&qr)[DK],
                                          const float (&u)[DK], float T, const int32_t *ex, int n_ex, float limit,
                                          float shift, int lane, int32_t &i1, float &d1, float &d2) {
  if constexpr (GL == 1)
    nn2<DK>(g, d, xg, qr, u, T, ex, n_ex, limit, shift, i1, d1, d2);
  else
    nn2_group<DK, GL>(g, d, xg, qr, u, T, ex, n_ex, limit, shift, lane, i1, d1, d2);
}

// Nearest nodes kept per cell (first candidates, and the list that answers
// most queries by itself).
template <int DK>
constexpr int knn_of() {
  return DK <= 2 ? 16 : (DK <= 3 ? 32 : (DK <= 4 ? 48 : 64));
}
static int knn_count(int d) { return d <= 2 ? 16 : (d <= 3 ? 32 : (d <= 4 ? 48 : 64)); }

// Per-cell list: the KN nearest nodes of x_i (excluding itself), nearest
// first, -1 past the end when n <= KN; their coordinates relative to x_i;
// and r2, the KN-th squared distance (+inf when the list holds every other
// node).  Every node outside the list is at least about sqrt(r2) from x_i:
// it was either rejected against a list bound that only decreases, or lies
// beyond the ring bound.  Ring search stopping once the ring bound exceeds
// the KN-th distance; the list is kept sorted by a fully unrolled insertion
// so it stays in registers.  Candidates below the list's current bound are
// first appended to a short per-lane buffer, which the whole wave merges
// into the lists at once when some lane's buffer is full (and before every
// stopping test): a wave then runs the insertion a few times per node
// instead of once for every candidate that any of its lanes accepts.  The
// insertions happen in candidate order, so the lists are the same.
struct KnnList {
  int32_t *ids;  // [n][KN]
  float *rel;    // [n][KN][d]
  float *r2;     // [n]
};

template <int DK>
__global__ __launch_bounds__(NT) void knn_kernel(const float *__restrict__ nodes, int64_t n, int d, GridView g,
                                                 KnnList out, const uint32_t *__restrict__ counters) {
  constexpr int KN = knn_of<DK>();
  // a non-finite node coordinate: no search at all (every ray is answered
  // NaN / -1 by the pass after the recheck)
  if (counters[CNT_BAD_NODES] != 0) return;
  // threads take the nodes in grid order, so a wave searches neighbouring cells
  const int64_t slot = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (slot >= n) return;
  const int64_t i = g.id[slot];
  float x[DK];
  int c[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    x[k] = k < d ? g.X[slot * d + k] : 0.f;
    int v = k < d ? (int)floorf(x[k] * (float)g.G) : 0;
    c[k] = v < 0 ? 0 : (v >= g.G ? g.G - 1 : v);
  }
  float dl[KN];
  int32_t il[KN];
#pragma unroll
  for (int s = 0; s < KN; ++s) {
    dl[s] = __builtin_inff();
    il[s] = -1;
  }
  constexpr int BUF = 4;  // 8 costs 8 more registers: 3 waves per SIMD at d = 3 instead of 4, 6% slower
  float bd[BUF];
  int32_t bi[BUF];
  int bc = 0;
  // merge the buffer into the sorted list, in append order
  auto flush = [&]() {
#pragma unroll
    for (int b = 0; b < BUF; ++b) {
      if (b < bc) {
        float dist = bd[b];
        int32_t node = bi[b];
        if (dist < dl[KN - 1]) {
#pragma unroll
          for (int s = 0; s < KN; ++s) {
            if (dist < dl[s]) {
              const float td = dl[s];
              const int32_t ti = il[s];
              dl[s] = dist;
              il[s] = node;
              dist = td;
              node = ti;
            }
          }
        }
      }
    }
    bc = 0;
  };
  for (int rho = 0; rho < g.G; ++rho) {
    if (rho >= 1) {
      flush();
      const float lb = fmaxf(0.f, (float)(rho - 1) * g.h - kRingSlack);
      if (lb * lb > dl[KN - 1]) break;
    }
    const int span = 2 * rho + 1;
    int o[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) o[k] = -rho;
    for (;;) {
      bool on_ring = false, inside = true;
      int64_t cell = 0;
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        if (k < d) {
          const int ck = c[k] + o[k];
          on_ring |= (o[k] == rho || o[k] == -rho);
          inside &= (ck >= 0 && ck < g.G);
          cell = cell * g.G + ck;
        }
      }
      if (on_ring && inside) {
        for (uint32_t p = g.start[cell]; p < g.start[cell + 1]; ++p) {
          int32_t node = g.id[p];
          if (node == (int32_t)i) continue;
          const float *xp = g.X + (int64_t)p * d;
          float dist = 0.f;
#pragma unroll
          for (int k = 0; k < DK; ++k) {
            if (k < d) {
              const float e = xp[k] - x[k];
              dist = __builtin_fmaf(e, e, dist);
            }
          }
          if (dist < dl[KN - 1]) {
#pragma unroll
            for (int b = 0; b < BUF; ++b) {
              if (b == bc) {
                bd[b] = dist;
                bi[b] = node;
              }
            }
            ++bc;
          }
          if (__any(bc == BUF)) flush();
        }
      }
      int k = d - 1;
      while (k >= 0) {
        if (++o[k] <= rho) break;
        o[k] = -rho;
        --k;
      }
      if (k < 0 || span == 1) break;
    }
  }
  flush();
#pragma unroll
  for (int s = 0; s < KN; ++s) {
    out.ids[i * KN + s] = il[s];
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) out.rel[(i * KN + s) * d + k] = il[s] >= 0 ? nodes[(int64_t)il[s] * d + k] - x[k] : 0.f;
    }
  }
  out.r2[i] = dl[KN - 1];
}

// Top-2 as nn2, over the cell's list only.
template <int DK, int KN, typename IP, typename FP>
__device__ void list_nn2(IP ids, FP rel, int d, const float (&u)[DK], float t, int32_t &i1,
                         float &d1, float &d2) {
  float qr[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) qr[k] = t * u[k];
  i1 = -1;
  d1 = d2 = __builtin_inff();
#pragma unroll 4
  for (int s = 0; s < KN; ++s) {
    // -1 marks the slots past the end (their coordinates are zero); the test
    // joins the value tests, with no branch around the next entry's loads
    const int32_t node = ids[s];
    float den = 0.f, dist = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {
        const float ek = rel[s * d + k];
        den = __builtin_fmaf(u[k], ek, den);
        const float e = qr[k] - ek;
        dist = __builtin_fmaf(e, e, dist);
      }
    }
    if (!((node >= 0) & (den > 0.f))) continue;
    if (dist < d1 || (dist == d1 && node < i1)) {
      d2 = d1;
      d1 = dist;
      i1 = node;
    } else if (dist < d2) {
      d2 = dist;
    }
  }
}

// Whether the cell's list answers a query at q = x_i + t u exactly as the
// grid would.  Only nodes with squared distance up to dmax = limit +
// gap_tol(limit, 2 limit) can change nn2's answer or its certificate (a
// farther node exceeds ref + gap_tol(ref, .) for ref <= limit, given
// shift < sqrt(limit) / 32); they lie within t + sqrt(dmax) of x_i, inside
// the list radius when this holds.
__device__ __forceinline__ bool list_covers(float t, float limit, float shift, float r2, int d) {
  const float dmax = limit + gap_tol(limit, 2.f * limit, shift, t, d);
  const float rr = t + sqrtf(dmax);
  return dmax <= 2.f * limit && 32.f * shift < sqrtf(limit) && rr * rr * (1.f + 0x1p-12f) < r2;
}

// Rays whose next query needs the grid, with their current candidate (-1:
// the exit-point test), handed from the list pass to the grid pass.
struct DeferQueue {
  int64_t *gid;     // [rays]
  int32_t *k;       // [rays]
  uint32_t *count;
};

// The RayCast of ray gid.  With GRID false the first candidate comes from
// the list, and a query the list cannot answer stops the ray: returns true
// with the current candidate in kdef, having written nothing.  With GRID
// true the ray resumes from kstart and such queries search the grid, by a
// group of GL lanes (all alike; lane 0 writes).  UNI: every active lane of
// the wave casts a ray of the same cell, whose list is then read through the
// constant address space with a wave-uniform address (scalar loads, shared
// by the wave) instead of one vector load per list entry and coordinate.
template <int DK, bool GRID, int GL = 1, bool UNI = false>
__device__ bool cast_ray(const CellScanArgs &a, const GridView &g, const KnnList &kl, int64_t gid,
                         int32_t kstart, int32_t &kdef, uint32_t &calls, uint32_t &grid_calls, int lane = 0) {
  constexpr int KN = knn_of<DK>();
  const int d = DK <= 4 ? DK : a.d;  // instances 2, 3 and 4 serve only their own d
  const int64_t cell = UNI ? (int64_t)__builtin_amdgcn_readfirstlane((int)(gid / a.R)) : gid / a.R;
  float xi[DK], u[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    xi[k] = k < d ? a.nodes[cell * d + k] : 0.f;
    u[k] = k < d ? a.dirs[gid * d + k] : 0.f;
  }
  // exit through the cube
  float tbox = __builtin_inff();
  int face = -1;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    if (k < d && u[k] != 0.f) {
      const float hk = u[k] > 0.f ? 1.f - xi[k] : xi[k];
      const float tk = hk / fabsf(u[k]);
      if (tk < tbox) {
        tbox = tk;
        face = 2 * k + (u[k] > 0.f ? 1 : 0);
      }
    }
  }
  using IP = typename std::conditional<UNI, const __attribute__((address_space(4))) int32_t *, const int32_t *>::type;
  using FP = typename std::conditional<UNI, const __attribute__((address_space(4))) float *, const float *>::type;
  const IP lids = (IP)(kl.ids + cell * KN);
  const FP lrel = (FP)(kl.rel + cell * KN * d);
  const float r2 = *(FP)(kl.r2 + cell);
  if (*g.outside) {  // the grid does not bound every node: settle in FP64
    if (lane != 0) return false;
    if (a.flag_list) {
      const uint32_t pos = atomicAdd(&a.counters[CNT_FLAGGED], 1u);
      a.flag_list[pos] = gid | a.flag_tag;
    }
    a.t_out[gid] = tbox;
    a.idx_out[gid] = -1;
    a.st_out[gid] = VG_ST_NEAR_TIE | VG_ST_SUSPECT;
    return false;
  }
  int32_t k = kstart;
  if (!GRID) {
    // first candidate: the eligible listed node with the smallest t_k =
    // num / (2 den) (grazing nodes, den <= |e| / 4096, are left out; their
    // t_k is large anyway).  Division-free: with den > 0 the order of the
    // t_k is that of the cross products; the best starts at the exit,
    // num / den = 2 tbox.  Any eligible node is a valid start.
    k = -1;
    float nb = 2.f * tbox, db = 1.f;
#pragma unroll 4
    for (int s = 0; s < KN; ++s) {
      const int32_t ks = lids[s];  // -1 past the end (see list_nn2)
      float num = 0.f, den = 0.f;
#pragma unroll
      for (int q2 = 0; q2 < DK; ++q2) {
        if (q2 < d) {
          const float e = lrel[s * d + q2];
          num = __builtin_fmaf(e, e, num);
          den = __builtin_fmaf(u[q2], e, den);
        }
      }
      if ((ks >= 0) & (den > 0.f) & (den * den > 0x1p-24f * num) & (num * db < nb * den)) {
        nb = num;
        db = den;
        k = ks;
      }
    }
  }
  bool flag = false;
  uint8_t st = 0;
  int32_t j = -1;
  float t = tbox;
  int32_t i1 = -1;
  float d1 = __builtin_inff(), d2 = __builtin_inff();
  if (face < 0) {
    flag = true;  // zero direction
    k = -1;
  } else if (k < 0) {
    float di = 0.f;  // squared distance of x_i to the exit point
#pragma unroll
    for (int q2 = 0; q2 < DK; ++q2) {
      const float e = tbox * u[q2];
      di = __builtin_fmaf(e, e, di);
    }
    // tbox: one subtraction and one division
    const float shift = tbox * 0x1p-22f;
    const bool in_list = list_covers(tbox, di, shift, r2, d);
    if (!GRID && !in_list) {
      kdef = -1;
      return true;
    }
    if (in_list) {
      list_nn2<DK, KN>(lids, lrel, d, u, tbox, i1, d1, d2);
    } else {
      const int32_t self = (int32_t)cell;
      float qr[DK];
#pragma unroll
      for (int q2 = 0; q2 < DK; ++q2) qr[q2] = tbox * u[q2];
      nn2_lanes<DK, GL>(g, d, xi, qr, u, tbox, &self, 1, di, shift, lane, i1, d1, d2);
      ++grid_calls;
    }
    ++calls;
    if (i1 == kGaveUp) {
      flag = true;
      st |= VG_ST_SUSPECT;
      j = -2 - face;
    } else if (i1 < 0 || d1 > di) {
      j = -2 - face;  // the exit point lies in cell i
      if (i1 >= 0 && !(d1 - di > gap_tol(d1, di, shift, tbox, d))) flag = true;
    } else {
      k = i1;
    }
  }
  if (k >= 0) {
    int it = 0;
    float shift = 0.f;
    for (; it < kMaxIter; ++it) {
      const float *xk = a.nodes + (int64_t)k * d;
      float ek[DK];
      float num = 0.f, den = 0.f;
#pragma unroll
      for (int q2 = 0; q2 < DK; ++q2) {
        ek[q2] = q2 < d ? xk[q2] - xi[q2] : 0.f;
        num = __builtin_fmaf(ek[q2], ek[q2], num);
        den = __builtin_fmaf(u[q2], ek[q2], den);
      }
      t = num / (2.f * den);
      // relative error of t: (d + 2) ulps of num, (d + 1) |e| / den ulps of
      // den (its cancellation), one of the division
      shift = t * ((float)(d + 3) + (float)(d + 1) * sqrtf(num) / den) * 0x1p-24f;
      float dk = 0.f;  // the candidate's own node: nothing farther matters
#pragma unroll
      for (int q2 = 0; q2 < DK; ++q2) {
        const float e = t * u[q2] - ek[q2];
        dk = __builtin_fmaf(e, e, dk);
      }
      const bool in_list = list_covers(t, dk, shift, r2, d);
      if (!GRID && !in_list) {
        kdef = k;
        return true;
      }
      if (in_list) {
        list_nn2<DK, KN>(lids, lrel, d, u, t, i1, d1, d2);
      } else {
        const int32_t self = (int32_t)cell;
        float qr[DK];
#pragma unroll
        for (int q2 = 0; q2 < DK; ++q2) qr[q2] = t * u[q2];
        nn2_lanes<DK, GL>(g, d, xi, qr, u, t, &self, 1, dk, shift, lane, i1, d1, d2);
        ++grid_calls;
      }
      ++calls;
      if (i1 == k) break;
      if (i1 < 0) break;  // k itself is eligible, so only through NaN
      k = i1;
    }
    j = k;
    if (it == kMaxIter || i1 != k) {
      flag = true;
      st |= VG_ST_SUSPECT;
    }
    // runner-up within rounding
    if (d2 < __builtin_inff() && !(d2 - d1 > gap_tol(d2, d1, shift, t, d))) flag = true;
    // a nearly grazing winner: its eligibility may hinge on rounding
    float den = 0.f, nrm = 0.f;
    const float *xj = a.nodes + (int64_t)j * d;
#pragma unroll
    for (int q2 = 0; q2 < DK; ++q2) {
      if (q2 < d) {
        const float e = xj[q2] - xi[q2];
        den = __builtin_fmaf(u[q2], e, den);
        nrm = __builtin_fmaf(e, e, nrm);
      }
    }
    if (!(den > (1.f / 4096.f) * sqrtf(nrm))) {
      flag = true;
      st |= VG_ST_SUSPECT;
    }
    t = reeval_cell<DK>(xi, xj, u, d);
    if (!(t <= tbox)) {  // the face is nearer after all: settle it in FP64
      flag = true;
    }
  }
  if (j <= -2) t = tbox;
  if (lane != 0) return false;
  if (flag && a.flag_list) {
    st |= VG_ST_NEAR_TIE;
    const uint32_t pos = atomicAdd(&a.counters[CNT_FLAGGED], 1u);
    a.flag_list[pos] = gid | a.flag_tag;
  }
  a.t_out[gid] = t;
  a.idx_out[gid] = j;
  a.st_out[gid] = st;
  return false;
}

// Sums the block's query counts into nn_calls[0] (all) and [1] (grid).
__device__ __forceinline__ void add_calls(unsigned int *block_calls, uint32_t calls, uint32_t grid_calls,
                                          unsigned long long *nn_calls) {
  if (calls) atomicAdd(&block_calls[0], calls);
  if (grid_calls) atomicAdd(&block_calls[1], grid_calls);
  __syncthreads();
  if (threadIdx.x < 2 && nn_calls) atomicAdd(nn_calls + threadIdx.x, (unsigned long long)block_calls[threadIdx.x]);
}

// List pass: one thread per ray; rays that need the grid are appended to the
// queue (one atomic per wave).
template <int DK>
__global__ __launch_bounds__(NT) void incircle_list_kernel(CellScanArgs a, GridView g, KnnList kl, DeferQueue dq,
                                                           unsigned long long *nn_calls) {
  // once per workgroup: the grid strides over the rays (a check at the start
  // of each of 2.5e5 short workgroups cost 1.7 ms of a 14.6 ms d=3 step)
  if (a.counters[CNT_BAD_NODES] != 0) return;  // see knn_kernel
  __shared__ unsigned int block_calls[2];
  if (threadIdx.x < 2) block_calls[threadIdx.x] = 0;
  __syncthreads();
  uint32_t calls = 0, grid_calls = 0;
  const int64_t total = a.n * a.R;
  for (int64_t base = (int64_t)blockIdx.x * NT; base < total; base += (int64_t)gridDim.x * NT) {
    const int64_t gid = base + threadIdx.x;
    bool defer = false;
    int32_t kdef = -1;
    const bool live = gid < total;
    // whether the wave's rays all belong to one cell (64 | R, or a cell boundary outside the wave)
    const int cell0 = __builtin_amdgcn_readfirstlane((int)(gid / a.R));
    const bool one_cell = __all(!live || gid / a.R == cell0);
    if (live) {
      if (one_cell)
        defer = cast_ray<DK, false, 1, true>(a, g, kl, gid, -1, kdef, calls, grid_calls);
      else
        defer = cast_ray<DK, false>(a, g, kl, gid, -1, kdef, calls, grid_calls);
    }
    const unsigned long long mask = __ballot(defer);
    if (mask) {
      const int lane = (int)__lane_id();
      const int leader = __ffsll((long long)mask) - 1;
      uint32_t qbase = 0;
      if (lane == leader) qbase = atomicAdd(dq.count, (uint32_t)__popcll(mask));
      qbase = __shfl(qbase, leader);
      if (defer) {
        const uint32_t pos = qbase + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        dq.gid[pos] = gid;
        dq.k[pos] = kdef;
      }
    }
  }
  add_calls(block_calls, calls, grid_calls, nn_calls);
}

// Grid pass over the queued rays, kRayLanes lanes per ray (grid-stride over
// the queue's count).
template <int DK>
__global__ __launch_bounds__(NT) void incircle_grid_kernel(CellScanArgs a, GridView g, KnnList kl, DeferQueue dq,
                                                           unsigned long long *nn_calls) {
  if (a.counters[CNT_BAD_NODES] != 0) return;  // see knn_kernel
  __shared__ unsigned int block_calls[2];
  if (threadIdx.x < 2) block_calls[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t cnt = *dq.count;
  const uint32_t gt = blockIdx.x * NT + threadIdx.x;
  const int lane = (int)(gt % kRayLanes);
  const uint32_t stride = gridDim.x * (NT / kRayLanes);
  uint32_t calls = 0, grid_calls = 0;
  for (uint32_t q = gt / kRayLanes; q < cnt; q += stride) {
    int32_t kd;
    (void)cast_ray<DK, true, kRayLanes>(a, g, kl, dq.gid[q], dq.k[q], kd, calls, grid_calls, lane);
  }
  if (lane != 0) calls = grid_calls = 0;
  add_calls(block_calls, calls, grid_calls, nn_calls);
}

// General rays (vg_raycast, the exhaustive search's edge rays): Algorithm 1
// from the origin x, or from InitialHeuristic's point when asked for and
// |eta| >= 2 (it projects x onto the hyperplane through x_g orthogonal to u,
// then walks the height r / sqrt((|eta|-1)(|eta|+1)) of a regular simplex
// over the face of radius r along u; the point stays on the ray's line).
// Everything is relative to the ray's generator x_g (an FP64 origin is made
// relative in FP64).  The first nn call gives the first candidate i; then
// t = (|r - x_i|^2 - |r - x_g|^2) / (2 u.(x_i - x_g)), r' = r + t u,
// j = nn(r'), until j = i.  The certificate is the one of the Monte-Carlo
// rays (gap of the two nearest eligible nodes at r' against their FP32
// error); uncertain, capped, grazing and no-hit rays go to the FP64 recheck.
// t* from the origin is then re-evaluated in FP64 from eq. (t).
// A group of GL lanes runs each ray: they share its queries (nn2_group) and
// compute everything else alike; lane 0 writes the results.
template <int DK, int GL>
__device__ void incircle_ray(const RayScanArgs &a, const GridView &g, int heuristic, int64_t ray, int lane,
                             uint32_t &calls) {
  const int d = a.d;
  const int32_t gidx = a.gen[ray];
  if (gidx < 0 || gidx >= a.n) {  // invalid generator index: report, skip
    if (lane == 0) {
      a.t_out[ray] = __builtin_nanf("");
      a.idx_out[ray] = -1;
      a.st_out[ray] = VG_ST_SUSPECT;
    }
    return;
  }
  if (*g.outside) {  // the grid does not bound every node: settle in FP64
    if (lane != 0) return;
    if (a.flag_list) {
      const uint32_t pos = atomicAdd(&a.counters[CNT_FLAGGED], 1u);
      a.flag_list[pos] = ray | a.flag_tag;
    }
    a.t_out[ray] = __builtin_inff();
    a.idx_out[ray] = -1;
    a.st_out[ray] = VG_ST_NEAR_TIE | VG_ST_SUSPECT;
    return;
  }
  const int32_t *ex = a.n_excl > 0 ? a.excl + ray * a.n_excl : nullptr;
  int n_eta = 0;  // members of eta (entries past the nodes are padding)
  for (int e = 0; e < a.n_excl; ++e) n_eta += (ex[e] >= 0 && ex[e] < a.n);
  float xg[DK], u[DK], r0[DK], r[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    if (k < d) {
      xg[k] = a.nodes[(int64_t)gidx * d + k];
      r0[k] = a.o64 ? (float)(a.o64[ray * d + k] - (double)xg[k]) : a.o32[ray * d + k] - xg[k];
      u[k] = a.u64 ? (float)a.u64[ray * d + k] : a.u32[ray * d + k];
    } else {
      xg[k] = u[k] = r0[k] = 0.f;
    }
    r[k] = r0[k];
  }
  float r0n = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) r0n = __builtin_fmaf(r0[k], r0[k], r0n);
  r0n = sqrtf(r0n);
  if (heuristic && n_eta >= 2) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) s = __builtin_fmaf(u[k], -r[k], s);
#pragma unroll
    for (int k = 0; k < DK; ++k) r[k] = __builtin_fmaf(s, u[k], r[k]);
    float rad = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) rad = __builtin_fmaf(r[k], r[k], rad);
    const float hh = sqrtf(rad) / sqrtf((float)((n_eta - 1) * (n_eta + 1)));
#pragma unroll
    for (int k = 0; k < DK; ++k) r[k] = __builtin_fmaf(hh, u[k], r[k]);
  }
  float rn = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) rn = __builtin_fmaf(r[k], r[k], rn);
  rn = sqrtf(rn);
  // the start point's own error (origin rounding, the heuristic's steps)
  const float shift0 = (2.f * r0n + 4.f * rn) * 0x1p-24f;
  int32_t i1;
  float d1, d2;
  nn2_group<DK, GL>(g, d, xg, r, u, rn, ex, a.n_excl, __builtin_inff(), shift0, lane, i1, d1, d2);
  ++calls;
  bool flag = a.force_all != 0;
  uint8_t st = 0;
  int32_t j = -1;
  double t64 = __builtin_inf();
  if (i1 == kGaveUp) {  // the FP64 recheck settles it
    flag = true;
    st |= VG_ST_SUSPECT;
  }
  if (i1 >= 0) {
    int32_t k = i1;
    int it = 0;
    float shift = shift0;
    float rp[DK];
    float rpn = 0.f;
    for (; it < kMaxIter; ++it) {
      const float *xk = a.nodes + (int64_t)k * d;
      float ek[DK];
      float num = 0.f, den = 0.f, en = 0.f;
#pragma unroll
      for (int q = 0; q < DK; ++q) {
        ek[q] = q < d ? xk[q] - xg[q] : 0.f;
        // |r - e|^2 - |r|^2 = e.(e - 2 r)
        num = __builtin_fmaf(ek[q], ek[q] - 2.f * r[q], num);
        den = __builtin_fmaf(u[q], ek[q], den);
        en = __builtin_fmaf(ek[q], ek[q], en);
      }
      const float t = num / (2.f * den);
      rpn = 0.f;
#pragma unroll
      for (int q = 0; q < DK; ++q) {
        rp[q] = __builtin_fmaf(t, u[q], r[q]);
        rpn = __builtin_fmaf(rp[q], rp[q], rpn);
      }
      rpn = sqrtf(rpn);
      // error of r': the start point's, then t's (num = e.(e - 2r) carries
      // (d+2) |e| (|e| + 2|r|) ulps, den (d+1) |e| ulps of t den, one
      // division), then the rounding of r + t u
      const float el = sqrtf(en);
      shift = shift0 + ((float)(d + 2) * el * (el + 2.f * rn) / (2.f * den) +
                        fabsf(t) * ((float)(d + 1) * el / den + 2.f) + rpn) * 0x1p-24f;
      float dk = 0.f;
#pragma unroll
      for (int q = 0; q < DK; ++q) {
        const float e = rp[q] - ek[q];
        dk = __builtin_fmaf(e, e, dk);
      }
      nn2_group<DK, GL>(g, d, xg, rp, u, rpn, ex, a.n_excl, dk, shift, lane, i1, d1, d2);
      ++calls;
      if (i1 == k) break;
      if (i1 < 0) break;  // k itself is eligible, so only through NaN
      k = i1;
    }
    j = k;
    if (it == kMaxIter || i1 != k) {
      flag = true;
      st |= VG_ST_SUSPECT;
    }
    if (d2 < __builtin_inff() && !(d2 - d1 > gap_tol(d2, d1, shift, rpn, d))) flag = true;
    // the winner's t from the origin, eq. (t) relative to x_g, in FP64
    const float *xj = a.nodes + (int64_t)j * d;
    double num = 0.0, den = 0.0, nrm = 0.0;
    for (int q = 0; q < d; ++q) {
      const double e = (double)xj[q] - (double)xg[q];
      // exact for an FP32 origin: the difference of two floats in FP64
      const double o = (a.o64 ? a.o64[ray * d + q] : (double)a.o32[ray * d + q]) - (double)xg[q];
      num += e * (e - 2.0 * o);
      den += (double)u[q] * e;
      nrm += e * e;
    }
    if (!(den > (1.0 / 4096.0) * sqrt(nrm))) {  // nearly grazing winner
      flag = true;
      st |= VG_ST_SUSPECT;
    }
    t64 = num / (2.0 * den);
  }
  float t = (float)t64;
  if (a.clip) {
    float tb = __builtin_inff();
    int face = -1;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d && u[k] != 0.f) {
        const float xa = a.o64 ? (float)a.o64[ray * d + k] : a.o32[ray * d + k];
        const float h = u[k] > 0.f ? 1.f - xa : -xa;
        const float tk = h / u[k];
        if (tk < tb) {
          tb = tk;
          face = 2 * k + (u[k] > 0.f ? 1 : 0);
        }
      }
    }
    if (face >= 0) {
      if (!(fabsf(tb - t) > 0x1p-16f * fmaxf(fabsf(tb), fabsf(t)))) flag = true;  // face against node
      if (tb < t) {
        t = tb;
        j = -2 - face;
      }
    }
  }
  if (j == -1) {
    st |= VG_ST_NO_HIT;
    t = __builtin_inff();
    flag = true;
  }
  if (lane != 0) return;
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
__global__ __launch_bounds__(NT) void incircle_rays_kernel(RayScanArgs a, GridView g, int heuristic,
                                                           unsigned long long *nn_calls) {
  if (a.counters[CNT_BAD_NODES] != 0) return;  // see knn_kernel; once per workgroup (grid-stride)
  __shared__ unsigned int block_calls[2];
  if (threadIdx.x < 2) block_calls[threadIdx.x] = 0;
  __syncthreads();
  uint32_t calls = 0;
  // kRayLanes divides NT, so a ray's lanes stay together in every step
  const int64_t total = a.m * kRayLanes;
  for (int64_t base = (int64_t)blockIdx.x * NT; base < total; base += (int64_t)gridDim.x * NT) {
    const int64_t gt = base + threadIdx.x;
    const int64_t ray = gt / kRayLanes;
    const int lane = (int)(gt % kRayLanes);
    uint32_t c = 0;
    if (ray < a.m) incircle_ray<DK, kRayLanes>(a, g, heuristic, ray, lane, c);
    if (lane == 0) calls += c;
  }
  add_calls(block_calls, calls, calls, nn_calls);
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + NT - 1) / NT); }
// workgroups of the grid-stride ray kernels (several rounds of the chip's
// resident workgroups, so the tails balance)
constexpr unsigned kStrideBlocks = 8192;

}  // namespace

static int incircle_grid_size(int64_t n, int d) {
  // about two nodes per cell, at most 2^22 cells
  int G = (int)std::floor(std::pow((double)n / 2.0, 1.0 / d));
  G = std::max(G, 1);
  while (G > 1 && std::pow((double)G, d) > 4194304.0) --G;
  return G;
}


namespace {

// Bump allocator over a scratch block (256-byte aligned pieces).
struct Carve {
  char *p;
  template <typename T>
  T *take(size_t count) {
    T *q = reinterpret_cast<T *>(p);
    p += (count * sizeof(T) + 255) & ~size_t(255);
    return q;
  }
};

size_t grid_bytes(int64_t n, int d) {
  const int G = incircle_grid_size(n, d);
  int64_t cells = 1;
  for (int k = 0; k < d; ++k) cells *= G;
  size_t tmp = 0;
  (void)hipcub::DeviceScan::InclusiveSum(nullptr, tmp, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                          (int)(cells + 1));
  // cell_of, ids [n] i32; Xs [n][d] f32; counts, start, cursor [cells + 1];
  // outside flag; scan temp
  return (size_t)n * 8 + (size_t)n * d * 4 + 3 * (size_t)(cells + 1) * 4 + tmp + 8 * 256;
}

// Counting sort of the nodes into the grid's cells (grid_bytes of scratch).
hipError_t build_grid(const float *nodes, int64_t n, int d, int large_budget, Carve &cv, GridView &g,
                      hipStream_t s) {
  const int G = incircle_grid_size(n, d);
  int64_t cells = 1;
  for (int k = 0; k < d; ++k) cells *= G;
  int32_t *cell_of = cv.take<int32_t>((size_t)n);
  int32_t *ids = cv.take<int32_t>((size_t)n);
  float *Xs = cv.take<float>((size_t)n * d);
  uint32_t *counts = cv.take<uint32_t>((size_t)(cells + 1));
  uint32_t *start = cv.take<uint32_t>((size_t)(cells + 1));
  uint32_t *cursor = cv.take<uint32_t>((size_t)(cells + 1));
  uint32_t *outside = cv.take<uint32_t>(1);
  size_t tmp = 0;
  hipError_t e = hipcub::DeviceScan::InclusiveSum(nullptr, tmp, counts, start, (int)(cells + 1), s);
  if (e != hipSuccess) return e;
  void *tmpp = cv.take<char>(tmp);
  e = fill_u32(counts, 0u, cells + 1, s);
  if (e == hipSuccess) e = fill_u32(cursor, 0u, cells + 1, s);
  if (e == hipSuccess) e = fill_u32(outside, 0u, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grid_count_kernel, dim3(blocks_of(n)), dim3(NT), 0, s, nodes, n, d, G, cell_of, counts,
                     outside);
  // counts[0] = 0 and counts[c + 1] = size of cell c, so the inclusive scan
  // gives start[c] = nodes in cells before c (start[cells] = n)
  e = hipcub::DeviceScan::InclusiveSum(tmpp, tmp, counts, start, (int)(cells + 1), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grid_fill_kernel, dim3(blocks_of(n)), dim3(NT), 0, s, nodes, n, d, cell_of, start, cursor,
                     Xs, ids);
  e = hipGetLastError();
  // offsets of a full sweep: sum over the rings of the (2 rho + 1)^d offsets
  // the ring loop enumerates
  double sweep = 0.0;
  for (int rho = 0; rho < G && sweep <= (double)kFullSweep; ++rho) sweep += std::pow(2.0 * rho + 1.0, d);
  const int budget = sweep <= (double)kFullSweep ? (int)sweep : large_budget;
  g = GridView{Xs, ids, start, G, 1.f / (float)G, outside, budget};
  return e;
}

}  // namespace

size_t incircle_rays_scratch_bytes(int64_t n, int d) { return grid_bytes(n, d); }

size_t incircle_scratch_bytes(int64_t n, int d, int R) {
  // the grid; list ids [n][KN] i32, rel [n][KN][d] f32, r2 [n] f32; queue
  // gid [rays] i64, k [rays] i32, count
  const size_t kn = (size_t)knn_count(d);
  const size_t rays = (size_t)n * (size_t)R;
  return grid_bytes(n, d) + (size_t)n * kn * (d + 1) * 4 + (size_t)n * 4 + rays * 12 + 6 * 256;
}

hipError_t launch_incircle_rays(const RayScanArgs &a, void *scratch, int heuristic, unsigned long long *nn_calls,
                                hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  Carve cv{static_cast<char *>(scratch)};
  GridView g;
  hipError_t e = build_grid(a.nodes, a.n, a.d, kRayRingBudget, cv, g, s);
  if (e != hipSuccess) return e;
  const dim3 grid(std::min(blocks_of(a.m * kRayLanes), kStrideBlocks)), blk(NT);
  if (a.d <= 2)
    hipLaunchKernelGGL(incircle_rays_kernel<2>, grid, blk, 0, s, a, g, heuristic, nn_calls);
  else if (a.d <= 3)
    hipLaunchKernelGGL(incircle_rays_kernel<3>, grid, blk, 0, s, a, g, heuristic, nn_calls);
  else if (a.d <= 4)
    hipLaunchKernelGGL(incircle_rays_kernel<4>, grid, blk, 0, s, a, g, heuristic, nn_calls);
  else
    hipLaunchKernelGGL(incircle_rays_kernel<6>, grid, blk, 0, s, a, g, heuristic, nn_calls);
  return hipGetLastError();
}

hipError_t launch_incircle_cells(const CellScanArgs &a, void *scratch, unsigned long long *nn_calls,
                                 hipStream_t s) {
  const int64_t n = a.n;
  const int d = a.d;
  const int64_t rays = n * a.R;
  if (rays >= (int64_t(1) << 32)) return hipErrorInvalidValue;  // 32-bit queue and flag counters
  Carve cv{static_cast<char *>(scratch)};
  GridView g;
  hipError_t e = build_grid(a.nodes, n, d, kRingBudget, cv, g, s);
  if (e != hipSuccess) return e;
  const size_t kn = (size_t)knn_count(d);
  KnnList kl;
  kl.ids = cv.take<int32_t>((size_t)n * kn);
  kl.rel = cv.take<float>((size_t)n * kn * d);
  kl.r2 = cv.take<float>((size_t)n);
  DeferQueue dq;
  dq.gid = cv.take<int64_t>((size_t)rays);
  dq.k = cv.take<int32_t>((size_t)rays);
  dq.count = cv.take<uint32_t>(1);
  e = fill_u32(dq.count, 0u, 1, s);
  if (e != hipSuccess) return e;
  const dim3 grid(std::min(blocks_of(rays), kStrideBlocks)), blk(NT);
  // the grid pass strides over the queue, whose length only the device knows
  const dim3 grid2(std::min<unsigned>(blocks_of(rays * kRayLanes), 16384u));
#define VG_INCIRCLE_LAUNCH(DKV)                                                                          \
  hipLaunchKernelGGL(knn_kernel<DKV>, dim3(blocks_of(n)), blk, 0, s, a.nodes, n, d, g, kl, a.counters); \
  hipLaunchKernelGGL(incircle_list_kernel<DKV>, grid, blk, 0, s, a, g, kl, dq, nn_calls);               \
  hipLaunchKernelGGL(incircle_grid_kernel<DKV>, grid2, blk, 0, s, a, g, kl, dq, nn_calls)
  if (d <= 2) {
    VG_INCIRCLE_LAUNCH(2);
  } else if (d <= 3) {
    VG_INCIRCLE_LAUNCH(3);
  } else if (d <= 4) {
    VG_INCIRCLE_LAUNCH(4);
  } else {
    VG_INCIRCLE_LAUNCH(6);
  }
#undef VG_INCIRCLE_LAUNCH
  return hipGetLastError();
}

}  // namespace vg
