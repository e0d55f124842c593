// Monte-Carlo RayCast of every cell on MFMA (gfx950): FP32 and split BF16x3.
//
// A ray of cell i starts at the generator x_i with eta = {i} (Algorithm 3),
// so eq. (t) reads t_r = |r - x_i|^2 / (2 u.(r - x_i)).  Inverting the nodes
// about x_i,  r~ = (r - x_i) / |r - x_i|^2,  gives  1 / (2 t_r) = u . r~,
// and the half-space restriction u.(r - x_i) > 0 becomes u . r~ > 0.  So
//     t* = 1 / (2 max_r u . r~)
// and the whole candidate scan of a cell is one dense contraction
// S = R~ . U^T (nodes x directions, K = d) with a max/argmax epilogue: no
// division, no mask, no cancellation between |r|^2 and x.r.  The faces of
// the cube are the mirror images of x_i and enter the same max in closed
// form: face x_k = 1 gives u_k / (2 (1 - x_k)), face x_k = 0 gives
// -u_k / (2 x_k).
//
// Work decomposition: one workgroup per (cell, chunk of RW rays).  Each wave
// owns C column blocks of 32 rays and keeps their directions as the MFMA B
// operand for the whole scan.  Nodes stream through LDS in chunks of one node
// per thread; every thread builds the inverted coordinates of its node
// (the X.R^T part of the scan, once per cell and node) and the waves then run
// v_mfma_f32_32x32x2_f32 over 32-node blocks.  Output layout of that MFMA:
// lane l holds column l%32 (one ray) and rows 8*(i/4) + 4*(l/32) + i%4 of
// register i, so the max over a lane's 16 values is register-local.
//
// Epilogue: per lane a running (best, second, argmax).  A 16-value block
// whose max does not exceed the lane's second best cannot change anything
// (fast path: an integer v_max3 tree over the bit patterns and one compare;
// best and second are never negative, and non-negative floats order like
// their bit patterns); a block max between second and best only becomes the
// new second; only a block holding a new best runs the exact top-2 update of
// its 16 values (v_max/v_med3 on the bit patterns) and the argmax search.
// A non-finite accumulator value (possible only next to a near-duplicate
// node, whose cell the certificate flags wholesale) makes best or second NaN,
// which the certificate's comparison also sends to the FP64 recheck.
//
// Near-tie certificate: with |u| = 1 the FP32 value of u.r~ is within
// (2d+4) 2^-24 |r~| of the exact one, and |r~| <= 1/nn_i (nn_i = distance to
// the nearest other node), so a gap above 2 (2d+4) 2^-24 / nn_i certifies the
// argmax.  Rays below max(kappa / nn_i, tau_rel * best) are queued for the
// FP64 recheck.  The winner's t* is re-evaluated from its two points in
// double-float arithmetic (error-free transformations), about FP32 rounding.
#pragma once

#include "vg_dfloat.h"
#include "vg_internal.h"
#include "vg_philox.h"

namespace vg {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int imax3(int a, int b, int c) { return max(max(a, b), c); }
// Maximum of the 16 values' bit patterns as signed integers: for a maximum
// >= +0 it is the bit pattern of the float maximum; otherwise it is negative.
__device__ __forceinline__ int max16_bits(const f32x16 &v) {
  int b[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) b[i] = __float_as_int(v[i]);
  const int m1 = imax3(b[0], b[1], b[2]), m2 = imax3(b[3], b[4], b[5]);
  const int m3 = imax3(b[6], b[7], b[8]), m4 = imax3(b[9], b[10], b[11]);
  const int m5 = imax3(b[12], b[13], b[14]);
  return max(imax3(m1, m2, m3), imax3(m4, m5, b[15]));
}

// Top-2 update of one lane with the 16 accumulator values of a 32x32 block.
// The argmax is kept encoded as (32-row block << 4) | register (decoded by
// decode_row), so the update needs no per-row index arithmetic.
//
// With m the block's maximum: a block with m <= second changes nothing; one
// with second < m <= best only raises second to m (every value of the block
// is <= best); only a block with m > best needs the exact running top-2 over
// its 16 values (prefix maximum and median-of-three) and the argmax, the
// lowest register that holds the new best.  The wave takes a branch when any
// of its lanes needs it, so the common middle case costs one instruction.
// All of it runs on the bit patterns: with best >= second >= +0, signed
// integer max and median order them as the floats (a negative value is
// below both and never enters).
__device__ __forceinline__ int imed3(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

__device__ __forceinline__ void epilogue16(const f32x16 &acc, float &best, float &second,
                                           int &bidx, int blk16) {
  const int m = max16_bits(acc);
  const int bb = __float_as_int(best), sb = __float_as_int(second);
  if (m > sb) {
    if (m > bb) {
      int v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = __float_as_int(acc[i]);
      int b = bb, s = sb;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        s = imed3(v[i], b, s);
        b = max(b, v[i]);
      }
      int idx = 15;
#pragma unroll
      for (int i = 14; i >= 0; --i) idx = (v[i] == m) ? i : idx;
      bidx = blk16 | idx;
      best = __int_as_float(m);
      second = __int_as_float(s);
    } else {
      second = __int_as_float(m);
    }
  }
}

// Node row of an encoded argmax held by `lane` (MFMA output layout above).
__device__ __forceinline__ int decode_row(int e, int lane) {
  if (e < 0) return e;
  return (e >> 4) * 32 + 8 * ((e & 15) >> 2) + (e & 3) + 4 * (lane >> 5);
}

// Coordinates of node r (zero beyond n or d).
template <int DK>
__device__ __forceinline__ void load_node(const float *__restrict__ nodes, int64_t n, int d,
                                          int64_t r, float (&x)[DK]) {
  const bool ok = r < n;
  const float *xr = nodes + (ok ? r : 0) * d;
#pragma unroll
  for (int k = 0; k < DK; ++k) x[k] = (ok && k < d) ? xr[k] : 0.f;
}

// Inverted coordinates r~ = (x_r - x_i)/|x_r - x_i|^2 of node r about x_i (zero
// for r = i, beyond n, and for a duplicate of x_i, which eq. (t) never makes
// eligible).  Returns |x_r - x_i|^2 (or +inf when not a node).
template <int DK>
__device__ __forceinline__ float invert_node(const float (&xr)[DK], const float (&xi)[DK],
                                             int64_t r, int64_t n, int64_t cell, float (&rt)[DK]) {
  if (r >= n || r == cell) {
#pragma unroll
    for (int k = 0; k < DK; ++k) rt[k] = 0.f;
    return __builtin_inff();
  }
  float n2 = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    rt[k] = xr[k] - xi[k];
    n2 = __builtin_fmaf(rt[k], rt[k], n2);
  }
  const float inv = n2 > 0.f ? __builtin_amdgcn_rcpf(n2) : 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) rt[k] *= inv;
  return n2;
}

// Node scanned as row r of `cell`: the row itself, or the r-th entry of the
// cell's candidate list.  Rows past the end and entries outside [0, n) give
// n, which load_node and invert_node treat as padding (a zero row never wins:
// the eligibility threshold is u.r~ > 0).
__device__ __forceinline__ int64_t row_node(const CellScanArgs &a, int64_t nb0, int64_t n_scan,
                                            int64_t r) {
  if (!a.nbr) return r;
  if (r >= n_scan) return a.n;
  const int32_t j = a.nbr[nb0 + r];
  return (j >= 0 && j < a.n) ? j : a.n;
}

// Chunks of the scan in visiting order: with the nodes in scan order
// (a.xs), the chunk that holds the cell's own node first, then alternately
// the next chunk above and below it; else 0, 1, 2, ...
// A value the whole workgroup holds alike (x_i, the cell's generator), moved
// to a scalar register: the scans keep their vector registers for the rays.
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

struct ChunkWalk {
  int lo, hi, nch;
  bool up;
  __device__ ChunkWalk(int first, int count) : lo(first - 1), hi(first + 1), nch(count), up(true) {}
  __device__ bool done() const { return lo < 0 && hi >= nch; }
  // the chunk after the current one, or -1
  __device__ int next() {
    if (lo < 0 && hi >= nch) return -1;
    const bool take_hi = (up && hi < nch) || lo < 0;
    up = !up;
    return take_hi ? hi++ : lo--;
  }
};

// Cross-lane reductions of non-negative floats (+inf allowed), on their bit
// patterns, which order like the values: DPP within each row of 16 lanes
// (quad permutes, half-row and row mirrors), then the four rows by readlane
// and scalar min/max.  A NaN pattern sorts above +inf.  Every source lane of
// these patterns lies in the row, so the move needs no old value: with
// bound_ctrl the compiler folds it into the min / max / add that uses it
// (v_max_u32_dpp and the like, one instruction per step instead of two).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t row_umin(uint32_t v) {
  v = min(v, dpp<0xb1>(v));      // quad_perm [1,0,3,2]
  v = min(v, dpp<0x4e>(v));      // quad_perm [2,3,0,1]
  v = min(v, dpp<0x141>(v));     // row_half_mirror
  return min(v, dpp<0x140>(v));  // row_mirror
}
__device__ __forceinline__ uint32_t row_umax(uint32_t v) {
  v = max(v, dpp<0xb1>(v));
  v = max(v, dpp<0x4e>(v));
  v = max(v, dpp<0x141>(v));
  return max(v, dpp<0x140>(v));
}
__device__ __forceinline__ uint32_t lane_u(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// Smallest value over the wave's 64 lanes (uniform).
__device__ __forceinline__ float wave_min(float v) {
  const uint32_t r = row_umin(__float_as_uint(v));
  return __uint_as_float(min(min(lane_u(r, 0), lane_u(r, 16)), min(lane_u(r, 32), lane_u(r, 48))));
}

// Largest value over the wave's 64 lanes (uniform).
__device__ __forceinline__ float wave_max(float v) {
  const uint32_t r = row_umax(__float_as_uint(v));
  return __uint_as_float(max(max(lane_u(r, 0), lane_u(r, 16)), max(lane_u(r, 32), lane_u(r, 48))));
}

// Value of lane l ^ 32.  v_permlane32_swap trades lanes 32-63 of its first
// operand with lanes 0-31 of its second: with both operands v, the first
// result holds lanes 0-31 of v in both halves and the second lanes 32-63.
__device__ __forceinline__ float partner32(float v, int lane) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(lane < 32 ? r[1] : r[0]);
}

// Upper bound on |u . r~| as any of the scans computes it, over the 32
// nodes of the caller's 32-lane block (|u| = 1 up to rounding, so
// |u . r~| <= |r~|; the factor 1 + 2^-12 covers the rounding of |r~|, of |u|
// and of the FP32 or split-BF16 dot product).  Stored by the block's last
// lane into bnd[block].
// Returns the bound (valid in the block's last lane).
template <int DK>
__device__ __forceinline__ float block_bound(const float (&rt)[DK], float *bnd, int tid) {
  float m2 = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) m2 = __builtin_fmaf(rt[k], rt[k], m2);
  uint32_t b = row_umax(__float_as_uint(__builtin_sqrtf(m2) * (1.f + 0x1p-12f)));
  // rows 1 and 3 take the maximum with rows 0 and 2 (row_bcast15)
  b = max(b, (uint32_t)__builtin_amdgcn_update_dpp((int)b, (int)b, 0x142, 0xa, 0xf, false));
  if ((tid & 31) == 31) bnd[tid >> 5] = __uint_as_float(b);
  return __uint_as_float(b);
}

// Adds the wave's count of evaluated 32x32 blocks to the call's counter.
__device__ __forceinline__ void count_blocks(const CellScanArgs &a, int blocks, int lane) {
  if (a.counters && lane == 0 && blocks)
    atomicAdd(reinterpret_cast<unsigned long long *>(a.counters + CNT_SCAN_BLOCKS), (unsigned long long)blocks);
}

// Sum over each row of 16 lanes (every lane of the row gets it).
__device__ __forceinline__ float row_fsum(float v) {
  v += __uint_as_float(dpp<0xb1>(__float_as_uint(v)));
  v += __uint_as_float(dpp<0x4e>(__float_as_uint(v)));
  v += __uint_as_float(dpp<0x141>(__float_as_uint(v)));
  return v + __uint_as_float(dpp<0x140>(__float_as_uint(v)));
}

// Centre and radius of the caller's 16-node half-block (its DPP row of 16
// lanes) in inverted coordinates: c = the mean of the 16 rows (any point
// would do; the mean keeps the radius small), rho = max |r~ - c| over the
// half-block, times 1 + 2^-12 for its rounding.  The row's first lane hands
// c to put(c, half) (which stores it as the scan's operand) and its last
// lane stores rho + 2^-11 B into rho[half], where B is the magnitude bound
// that lane holds from block_bound (its row's or its block's, both bounds
// on the half-block's |r~| and so on |c|), which covers the rounding of the
// dot products with c and with the nodes: then, for any ray, no computed
// u.r~ of the half-block exceeds the computed u.c plus rho[half].  Two
// halves bound a block more tightly than one centre, and their sums are the
// row sums the reduction forms first.
template <int DK, class Put>
__device__ __forceinline__ void block_centre(const float (&rt)[DK], float bb, float *rho, int d, int tid,
                                             Put &&put) {
  const int half = tid >> 4;
  float c[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) c[k] = k < d ? row_fsum(rt[k]) * (1.f / 16.f) : 0.f;
  float r2 = 0.f;
#pragma unroll
  for (int k = 0; k < DK; ++k) {
    const float e = rt[k] - c[k];
    r2 = __builtin_fmaf(e, e, r2);
  }
  const uint32_t r = row_umax(__float_as_uint(__builtin_sqrtf(r2) * (1.f + 0x1p-12f)));
  if ((tid & 15) == 0) put(c, half);
  if ((tid & 15) == 15) rho[half] = __uint_as_float(r) + bb * 0x1p-11f;
}

// Largest second-best value a ray holds: each lane keeps the top two of its
// half of the 32 node rows, the lane l ^ 32 those of the other half.
__device__ __forceinline__ float merged_second(float b, float s, int lane) {
  const float ob = partner32(b, lane), os = partner32(s, lane);
  return fmaxf(fmaxf(s, os), fminf(b, ob));
}

// Upper bound on |u . r~| over the nodes of scan-order chunk c (NB nodes, the
// 128-node boxes of the order pass): 1 / (distance from x_i to the boxes),
// with a factor 1 + 2^-10 above the block bounds' 1 + 2^-12, so the chunk
// that holds x_i's nearest node never falls below a bound taken from values
// of that chunk.  Uniform over the wave.
template <int NB, int DK>
__device__ __forceinline__ float chunk_bound(const CellScanArgs &a, const float (&xi)[DK], int c, int lane) {
  constexpr int GPC = NB / kOrderGroup;
  const int d = a.d;
  const int64_t g = (int64_t)c * GPC + lane;
  float b = 0.f;
  if (lane < GPC && g * kOrderGroup < a.n) {
    const float *box = a.aabb + g * 2 * d;
    float s2 = 0.f;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d) {
        const float gap = fmaxf(fmaxf(box[k] - xi[k], xi[k] - box[d + k]), 0.f);
        s2 = __builtin_fmaf(gap, gap, s2);
      }
    }
    b = s2 > 0.f ? __builtin_amdgcn_rsqf(s2) * (1.f + 0x1p-10f) : __builtin_inff();
  }
  return wave_max(b);
}

// The same bound for chunk c computed by one thread (no reduction).
template <int NB, int DK>
__device__ __forceinline__ float chunk_bound_thread(const CellScanArgs &a, const float (&xi)[DK], int c) {
  constexpr int GPC = NB / kOrderGroup;
  const int d = a.d;
  float b = 0.f;
#pragma unroll
  for (int j = 0; j < GPC; ++j) {
    const int64_t g = (int64_t)c * GPC + j;
    if (g * kOrderGroup < a.n) {
      const float *box = a.aabb + g * 2 * d;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < DK; ++k) {
        if (k < d) {
          const float gap = fmaxf(fmaxf(box[k] - xi[k], xi[k] - box[d + k]), 0.f);
          s2 = __builtin_fmaf(gap, gap, s2);
        }
      }
      b = fmaxf(b, s2 > 0.f ? __builtin_amdgcn_rsqf(s2) * (1.f + 0x1p-10f) : __builtin_inff());
    }
  }
  return b;
}

// Chunk bounds kept in LDS for the whole walk when the cloud has at most
// this many chunks (else evaluated one by one as the walk reaches them).
constexpr int kChunkTable = 2048;

// A chunk's table entry: its bound's bit pattern with the low 11 bits
// replaced by the chunk index (< kChunkTable), so that the entries sort like
// the bounds; key_bound rounds the bound back up to the end of its bucket
// (at most 2^-12 relative above the bound: still a bound).
__device__ __forceinline__ uint32_t chunk_key(float b, int c) {
  return (__float_as_uint(b) & ~(uint32_t)(kChunkTable - 1)) | (uint32_t)c;
}
__device__ __forceinline__ float key_bound(uint32_t key) {
  return __uint_as_float(min((key | (uint32_t)(kChunkTable - 1)) + 1u, 0x7f800000u));
}

// The loop over the chunks of NB nodes shared by the FP32 and BF16x3 scans.
// stage(rt) stores the calling thread's inverted node into the LDS tile;
// block(nb, blk16, skip) runs the column blocks cb of node block nb for
// which skip(cb) is false and returns how many it ran.  Returns the number of
// 32x32 blocks the wave evaluated.
//
// Index order (!SORTED, also the candidate lists): every chunk, every block.
// Scan order (SORTED): the cell's own chunk first, then outwards (ChunkWalk).
// Every bound below holds for |u| = 1 up to rounding; `prune` (uniform) says
// that every ray of the workgroup has such a direction, and without it
// nothing is skipped.  A node block is skipped for column block cb when its
// bound is below the smallest merged second best of cb's 32 rays (none of
// its values can enter a ray's top two: they are at most that second best,
// and an equal value would only make a tie the certificate flags anyway).
// A whole chunk is not even loaded
//  - when its box bound is below the smallest such value over the workgroup,
//    taken two chunks earlier from wsm (the slot of the same parity, written
//    after that chunk's second barrier, read before this chunk's first);
//  - (WIN) when no ray of the workgroup reaches the bound of its groups'
//    balls inverted about x_i: the walk is cut into windows of 32 groups
//    (32 / GPC chunks that pass the box bound); at a window's start every
//    wave computes u.c' for the 32 inverted centres c' with one product
//    chain per column block (window(cb, c'): lane l holds row l % 32's
//    centre), compares u.c' + e' with each
//    ray's merged second, and the workgroup ORs the waves' group masks
//    through wmask (two slots, alternating: a slot is rewritten only after
//    a later barrier all waves have passed).  A column block's own mask also
//    removes the node blocks of groups none of its rays reach.
// The ball of a group (centre c, radius r, holding every node of the group)
// inverted about x_i is the ball of centre c' = (c - x_i) / D and radius
// r / D, D = |c - x_i|^2 - r^2 > 0 (x_i outside), so u.r~ <= u.c' + r / D
// for |u| = 1.  With D >= 2^-8 |c - x_i|^2 its FP32 evaluation is within
// (d + 3) 2^-24 |c - x_i|^2 / D <= 2^-11.7 of D relative, c' and r / D within
// about 2^-10.9 of |c'| = |c - x_i| / D; e' = (r + 2^-8 |c - x_i|) / D covers
// these, the rounding of the inverted nodes and of the FP32 or split-BF16
// products with room to spare.  Closer groups (x_i inside or near the ball)
// are always needed.
template <int DK, int C, int NB, int WAVES, bool SORTED, bool CENTRES, bool WIN, bool BIG, class Stage,
          class Block, class Put, class Centres, class Window>
__device__ __forceinline__ int scan_chunks(const CellScanArgs &a, int64_t cell, const float (&xi)[DK],
                                           const float (&best)[C], const float (&second)[C], float &nn2,
                                           float *bnd, float *wsm, uint32_t *wmask, float *ctab, float *rho,
                                           int64_t nb0, int64_t n_scan, int rayw, bool prune, Stage &&stage,
                                           Block &&block, Put &&put, Centres &&centres, Window &&window) {
  static_assert(NB / 32 <= 32, "block masks are 32 bits");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int d = a.d;
  const int64_t n = a.n;
  int blocks = 0;
  float pre[DK];
  if constexpr (!SORTED) {
    // the coordinates of the next chunk's node are loaded one chunk ahead, so
    // their latency hides behind the MFMA loop of the current chunk
    load_node<DK>(a.nodes, n, d, row_node(a, nb0, n_scan, tid), pre);
    for (int64_t base = 0; base < n_scan; base += NB) {
      float rt[DK];
      nn2 = fminf(nn2, invert_node<DK>(pre, xi, row_node(a, nb0, n_scan, base + tid), n, cell, rt));
      load_node<DK>(a.nodes, n, d, row_node(a, nb0, n_scan, base + NB + tid), pre);
      __syncthreads();  // the previous chunk is consumed
      stage(rt);
      __syncthreads();
      const int64_t rem = n_scan - base;
      const int nblocks = rem >= NB ? NB / 32 : (int)((rem + 31) / 32);
      for (int nb = 0; nb < nblocks; ++nb)
        blocks += block(nb, (int)((base >> 5) + nb) << 4, [](int) { return false; });
    }
  } else {
    static_assert(NB % kOrderGroup == 0, "chunks hold whole groups");
    constexpr int GPC = NB / kOrderGroup;  // groups per chunk
    constexpr int WS = 32 / GPC;           // chunks per window
    constexpr uint32_t GMASK = (1u << GPC) - 1u;
    const int64_t self = a.rank[cell];
    const int c0 = (int)(self / NB);
    const int nch = (int)((n + NB - 1) / NB);
    ChunkWalk walk(c0, nch);
    // Every chunk's bound up front (they depend on x_i only), sorted from the
    // largest down: the walk then takes the chunks most likely to hold the
    // rays' winners first, so the thresholds rise sooner, and it ends at the
    // first chunk whose bound is below the workgroup's threshold (all later
    // ones are below it too).  The order decides only the speed.
    //
    // Clouds of more chunks than the table holds are launched on the BIG
    // instance: each entry is shared by S consecutive chunks and keyed by the
    // largest of their bounds; the walk takes the entries in that order and,
    // inside an entry, the chunks whose own bound reaches the threshold, and
    // it ends at the first entry whose key is below the threshold (its state
    // would cost the other instances registers).  The other instances, given
    // such a cloud, walk outwards from x_i's chunk in scan order, with each
    // bound computed as the walk reaches it.
    const bool table = !BIG && nch <= kChunkTable;
    const int S = BIG ? (nch + kChunkTable - 1) / kChunkTable : 1;  // chunks per entry
    const int nent = BIG ? (nch + S - 1) / S : nch;
    uint32_t *ckey = reinterpret_cast<uint32_t *>(ctab);
    if (BIG || table) {
      int p2 = 2;
      while (p2 < nent) p2 <<= 1;
      if constexpr (BIG) {
        for (int e = tid; e < p2; e += WAVES * 64) {
          uint32_t key = 0u;  // 0: after every entry
          if (e < nent) {
            float b = 0.f;
            const int c1 = min(e * S + S, nch);
            for (int c = e * S; c < c1; ++c) b = fmaxf(b, chunk_bound_thread<NB, DK>(a, xi, c));
            key = chunk_key(b, e);
          }
          ckey[e] = key;
        }
      } else {
        for (int c = tid; c < p2; c += WAVES * 64)
          ckey[c] = c < nch ? chunk_key(chunk_bound_thread<NB, DK>(a, xi, c), c) : 0u;  // 0: after every chunk
      }
      __syncthreads();  // uniform: table depends on n only
      // bitonic sort, descending
      for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int t = tid; t < p2 / 2; t += WAVES * 64) {
            const int i = 2 * t - (t & (j - 1));
            const uint32_t x = ckey[i], y = ckey[i + j];
            if ((x < y) == ((i & k) == 0)) {
              ckey[i] = y;
              ckey[i + j] = x;
            }
          }
          __syncthreads();
        }
      }
    }
    int spos = 0;  // table: next position in the sorted keys
    int enext = 0, eend = 0;  // BIG: chunks of the current entry not yet taken
    // the walk's next chunk other than x_i's own (-1: none left) and its
    // bound; BIG: only chunks whose bound reaches thr_now
    auto next_chunk = [&](float &bnd, float thr_now) -> int {
      if constexpr (BIG) {
        for (;;) {
          while (enext < eend) {
            const int c = enext++;
            if (c == c0) continue;
            bnd = chunk_bound<NB, DK>(a, xi, c, lane);
            if (bnd < thr_now) continue;
            return c;
          }
          if (spos >= nent) return -1;
          const uint32_t key = __builtin_amdgcn_readfirstlane(ckey[spos++]);
          if (key_bound(key) < thr_now) {  // so are the later entries
            spos = nent;
            return -1;
          }
          enext = (int)(key & (uint32_t)(kChunkTable - 1)) * S;
          eend = min(enext + S, nch);
        }
      }
      if (table) {
        while (spos < nch) {
          const uint32_t key = ckey[spos++];
          const int c = (int)(key & (uint32_t)(kChunkTable - 1));
          if (c == c0) continue;
          bnd = key_bound(key);
          return c;
        }
        return -1;
      }
      const int c = walk.next();
      if (c >= 0) bnd = chunk_bound<NB, DK>(a, xi, c, lane);
      return c;
    };
    auto walk_done = [&]() {
      if constexpr (BIG) return spos >= nent && enext >= eend;
      return table ? spos >= nch : walk.done();
    };
    // a chunk's bound fell below the threshold: in the sorted walk so does
    // every later one (BIG: such chunks are skipped inside next_chunk)
    auto below = [&]() {
      if (table) spos = nch;
    };
    // per column block, the value a ray's bound must reach: its merged second
    // best; +inf on lanes of padding rays (ray >= R, zero direction), which
    // constrain nothing; 0 without prune (no bound is below it)
    auto floors = [&](float (&ms)[C]) {
#pragma unroll
      for (int cb = 0; cb < C; ++cb) {
        const float m = merged_second(best[cb], second[cb], lane);
        ms[cb] = !prune ? 0.f : (rayw + cb * 32 + (lane & 31) < a.R ? m : __builtin_inff());
      }
    };
    const float *ball = a.aabb + order_groups(n) * 2 * d;
    uint32_t wq = 0u;       // window slots not yet visited
    int slot_chunk = -1;    // lane s < WS: the chunk of window slot s
    float slot_bnd = 0.f;   // and its bound
    uint32_t gneed[C];      // bit j: window group j reaches some ray of cb
    int wpar = 0;
    // backoff of the window test: after a test that rejects fewer than an
    // eighth of its chunks the next `idle` windows are taken untested (the
    // test costs about as much as staging a chunk per column block; where
    // the balls rarely separate, as in uniform clouds of d >= 10, it would
    // only cost)
    int idle = 0, untested = 0;
    // A new window: its chunks (in walk order, past the box bound) and the
    // mask of the slots the workgroup needs.  Uniform; one barrier.
    auto refill = [&](float thr_now) -> uint32_t {
      int cnt = 0, my_chunk = -1;  // row j = lane % 32 is group j % GPC of slot j / GPC
      slot_chunk = -1;
      while (cnt < WS) {
        float b;
        const int c = next_chunk(b, thr_now);
        if (c < 0) break;
        if (b < thr_now) {
          if (table) {
            below();
            break;
          }
          continue;
        }
        if ((lane & 31) / GPC == cnt) my_chunk = c;
        if (lane == cnt) {
          slot_chunk = c;
          slot_bnd = b;
        }
        ++cnt;
      }
      if (cnt == 0) return 0u;
      const uint32_t all_slots = cnt >= 32 ? ~0u : (1u << cnt) - 1u;
      if (!prune || untested > 0) {
        untested = untested > 0 ? untested - 1 : 0;
#pragma unroll
        for (int cb = 0; cb < C; ++cb) gneed[cb] = ~0u;
        return all_slots;
      }
      // lane row's group ball inverted about x_i: centre cp = (c - x_i) / D
      // and e' = (r + 2^-8 |c - x_i|) / D; cp = 0 without a group (e' = -inf:
      // never needed) or with x_i inside or near it (e' = +inf)
      float cp[DK], e = -__builtin_inff();
#pragma unroll
      for (int k = 0; k < DK; ++k) cp[k] = 0.f;
      const int64_t g = (int64_t)my_chunk * GPC + ((lane & 31) % GPC);
      if (my_chunk >= 0 && g < order_groups(n)) {
        const float *bp = ball + g * (d + 1);
        float s2 = 0.f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
          cp[k] = k < d ? bp[k] - xi[k] : 0.f;
          s2 = __builtin_fmaf(cp[k], cp[k], s2);
        }
        const float r = bp[d];
        const float D = __builtin_fmaf(-r, r, s2);
        if (D > s2 * 0x1p-8f && D < __builtin_inff()) {
          const float inv = 1.f / D;
#pragma unroll
          for (int k = 0; k < DK; ++k) cp[k] *= inv;
          e = __builtin_fmaf(0x1p-8f, __builtin_sqrtf(s2), r) * inv;
        } else {
#pragma unroll
          for (int k = 0; k < DK; ++k) cp[k] = 0.f;
          e = __builtin_inff();
        }
      }
      float ms[C];
      floors(ms);
      uint32_t wm = 0u;
#pragma unroll
      for (int cb = 0; cb < C; ++cb) {
        gneed[cb] = 0u;
        if (__ballot(ms[cb] < __builtin_inff()) == 0ull) continue;  // padding rays only
        // u.c' + e' (one more K step adds e' of each row: A = e' and B = 1 in
        // lane half 0, zero in half 1); register i of lane half h holds row
        // 8 (i / 4) + 4 h + i % 4
        const f32x16 uc = __builtin_amdgcn_mfma_f32_32x32x2f32(lane < 32 ? e : 0.f, lane < 32 ? 1.f : 0.f,
                                                               window(cb, cp), 0, 0, 0);
        uint32_t nd = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const uint64_t m = __ballot(!(uc[i] < ms[cb]));
          const int row = 8 * (i >> 2) + (i & 3);
          nd |= ((uint32_t)(m & 0xffffffffull) != 0u ? 1u : 0u) << row;
          nd |= ((uint32_t)(m >> 32) != 0u ? 1u : 0u) << (row + 4);
        }
        gneed[cb] = nd;
        wm |= nd;
      }
      if (lane == 0) wmask[wpar * WAVES + wave] = wm;
      __syncthreads();
      uint32_t all = 0u;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) all |= wmask[wpar * WAVES + w];
      wpar ^= 1;
      uint32_t q = 0u;
#pragma unroll
      for (int sl = 0; sl < WS; ++sl)
        if (sl < cnt && ((all >> (sl * GPC)) & GMASK)) q |= 1u << sl;
      if (8 * (cnt - __builtin_popcount(q)) < cnt) {
        idle = idle < 8 ? idle + 1 : 8;
        untested = idle;
      } else {
        idle = 0;
      }
      return q;
    };
    int64_t base = (int64_t)c0 * NB;
    float thr = 0.f;
    uint32_t cur_g[C];  // groups of the current chunk that reach a ray of cb
#pragma unroll
    for (int cb = 0; cb < C; ++cb) cur_g[cb] = GMASK;
    load_node<DK>(a.xs, n, d, base + tid, pre);
    for (int it = 0; base >= 0; ++it) {
      float rt[DK];
      nn2 = fminf(nn2, invert_node<DK>(pre, xi, base + tid, n, self, rt));
      if (it >= 2) {
        float t = wsm[(it & 1) * WAVES];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) t = fminf(t, wsm[(it & 1) * WAVES + w]);
        thr = t;
      }
      // the next chunk: the next slot of the window the workgroup needs (or
      // the walk's next chunk) whose box bound still reaches thr; its nodes
      // load while this chunk is staged and scanned
      int next = -1;
      uint32_t nxt_g[C];
#pragma unroll
      for (int cb = 0; cb < C; ++cb) nxt_g[cb] = GMASK;
      auto pop = [&]() {
        while (wq != 0u) {
          const int sl = __builtin_ctz(wq);
          wq &= wq - 1u;
          const int c = __builtin_amdgcn_readlane(slot_chunk, sl);
          if (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(slot_bnd), sl)) < thr) {
            if (table) {  // the later slots and chunks are below thr too
              wq = 0u;
              below();
            }
            continue;
          }
          next = c;
#pragma unroll
          for (int cb = 0; cb < C; ++cb) nxt_g[cb] = (gneed[cb] >> (sl * GPC)) & GMASK;
          return;
        }
      };
      if constexpr (WIN) {
        pop();
      } else {
        float b;
        next = next_chunk(b, thr);
        while (next >= 0 && b < thr) {
          if (table) {
            below();
            next = -1;
            break;
          }
          next = next_chunk(b, thr);
        }
      }
      if (next >= 0) load_node<DK>(a.xs, n, d, (int64_t)next * NB + tid, pre);
      __syncthreads();  // the previous chunk is consumed
      stage(rt);
      const float bb_own = block_bound<DK>(rt, bnd, tid);
      if constexpr (CENTRES) block_centre<DK>(rt, bb_own, rho, d, tid, put);
      if constexpr (WIN) {
        // window spent: the next windows are tested here, where rt is dead
        // (the test's registers do not add to it)
        if (next < 0) {
          while (next < 0 && !walk_done()) {
            wq = refill(thr);
            pop();
          }
          if (next >= 0) load_node<DK>(a.xs, n, d, (int64_t)next * NB + tid, pre);
        }
      }
      const int64_t nbase = next >= 0 ? (int64_t)next * NB : -1;
      __syncthreads();
      float smin[C], ms[C];
      float sall = __builtin_inff();
      floors(ms);
#pragma unroll
      for (int cb = 0; cb < C; ++cb) {
        smin[cb] = wave_min(ms[cb]);
        sall = fminf(sall, smin[cb]);
      }
      if (lane == 0) wsm[(it & 1) * WAVES + wave] = sall;
      const int64_t rem = n - base;
      const int nblocks = rem >= NB ? NB / 32 : (int)((rem + 31) / 32);
      // lane b < nblocks holds the bound of node block b
      const float lb = lane < nblocks ? bnd[lane] : 0.f;
      if (!(wave_max(lb) < sall)) {
        // run[cb] bit b: node block b for column block cb, by the magnitude
        // bound, the groups' balls (WIN) and the centre bound u.c + rho
        // (CENTRES) of some ray of cb
        uint32_t run[C], any = 0u;
#pragma unroll
        for (int cb = 0; cb < C; ++cb) {
          run[cb] = (uint32_t)__ballot(!(lb < smin[cb]) && lane < nblocks);
          if constexpr (WIN) {
            uint32_t gb = 0u;  // each group is kOrderGroup / 32 = 4 node blocks
#pragma unroll
            for (int gi = 0; gi < GPC; ++gi) gb |= ((cur_g[cb] >> gi) & 1u) ? 0xfu << (4 * gi) : 0u;
            run[cb] &= gb;
          }
          any |= run[cb];
        }
        if constexpr (CENTRES) {
          if (prune) {
            // rows 0 .. NB/16 - 1 of the centre product, the chunk's
            // half-blocks: register i of lane half h holds row
            // 8 (i / 4) + 4 h + i % 4, so registers 2q and 2q + 1 hold the
            // two halves of block 4 (q / 2) + 2 h + q % 2, whose bound is the
            // larger of theirs
            constexpr int NI = NB / 32;
            float eb[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) eb[i] = rho[8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)];
            any = 0u;
#pragma unroll
            for (int cb = 0; cb < C; ++cb) {
              if (run[cb] == 0u) continue;  // no block in reach (also padding rays only)
              const f32x16 uc = centres(cb);
              uint32_t nd = 0;
#pragma unroll
              for (int q = 0; q < NI / 2; ++q) {
                const float bm = fmaxf(uc[2 * q] + eb[2 * q], uc[2 * q + 1] + eb[2 * q + 1]);
                const uint64_t m = __ballot(!(bm < ms[cb]));
                const int blk = 4 * (q >> 1) + (q & 1);
                nd |= ((uint32_t)(m & 0xffffffffull) != 0u ? 1u : 0u) << blk;
                nd |= ((uint32_t)(m >> 32) != 0u ? 1u : 0u) << (blk + 2);
              }
              run[cb] &= nd;
              any |= run[cb];
            }
          }
        }
        while (any) {
          const int nb = __builtin_ctz(any);
          any &= any - 1u;
          blocks += block(nb, (int)((base >> 5) + nb) << 4, [&](int cb) { return !((run[cb] >> nb) & 1u); });
        }
      }
      base = nbase;
#pragma unroll
      for (int cb = 0; cb < C; ++cb) cur_g[cb] = nxt_g[cb];
    }
  }
  return blocks;
}

// Rays [r0, r0 + RW) of `cell` when a node coordinate of the call is not
// finite (the input check counted it): no answer, t = NaN, idx = -1.  The
// whole workgroup takes this path or none (the count is read by all).
template <int NT>
__device__ __forceinline__ bool item_bad_nodes(const CellScanArgs &a, int64_t cell, int r0, int RW) {
  if (!a.counters || a.counters[CNT_BAD_NODES] == 0) return false;
  const int nr = min(RW, a.R - r0);
  for (int r = threadIdx.x; r < nr; r += NT) {
    const int64_t gid = cell * a.R + r0 + r;
    a.t_out[gid] = __builtin_nanf("");
    a.idx_out[gid] = -1;
    a.st_out[gid] = VG_ST_BAD_INPUT;
  }
  if (threadIdx.x == 0 && nr > 0) atomicAdd(&a.counters[CNT_BAD_RAYS], (uint32_t)nr);
  return true;
}

// Merge the two lanes of each ray, add the cube faces, certify the gap,
// re-evaluate t* and write the ray results.
template <int C, int DK, int NT, bool GEN>
__device__ __forceinline__ void cell_finish(const CellScanArgs &a, const float (&xi)[DK],
                                            float (&best)[C], float (&second)[C], int (&bidx)[C],
                                            float nn2, float *red, int lane, int rayw,
                                            int64_t cell, int64_t nb0, int64_t n_scan) {
  const int d = a.d;
  const int R = a.R;
  // nearest-neighbour distance of x_i (for the error certificate)
  const int tid = threadIdx.x;
  red[tid] = nn2;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fminf(red[tid], red[tid + s]);
    __syncthreads();
  }
  const float nn = sqrtf(red[0]);

  // merge the two lanes that hold each ray (rows split by l/32)
#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    bidx[cb] = decode_row(bidx[cb], lane);
    const float ob = __shfl_xor(best[cb], 32);
    const float os = __shfl_xor(second[cb], 32);
    const int oi = __shfl_xor(bidx[cb], 32);
    const bool take = (ob > best[cb]) || (ob == best[cb] && oi >= 0 && (bidx[cb] < 0 || oi < bidx[cb]));
    const float other = take ? best[cb] : ob;
    if (take) {
      best[cb] = ob;
      bidx[cb] = oi;
    }
    second[cb] = fmaxf(fmaxf(second[cb], os), other);
  }
  if (lane >= 32) return;

#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    const int ray = rayw + cb * 32 + lane;
    if (ray >= R) continue;
    const int64_t gid = (int64_t)cell * R + ray;
    float u[DK];
    cell_dir<DK>(GEN ? nullptr : a.dirs, a.seed, cell, R, ray, d, u);
    // cube faces as mirror images of x_i
    float sbox = 0.f, tbox = __builtin_inff();
    int face = -1;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
      if (k < d && u[k] != 0.f) {
        const float h = u[k] > 0.f ? 1.f - xi[k] : xi[k];
        const float sk = fabsf(u[k]) / (2.f * h);
        if (sk > sbox) {
          sbox = sk;
          tbox = h / fabsf(u[k]);
          face = 2 * k + (u[k] > 0.f ? 1 : 0);
        }
      }
    }
    float s1 = best[cb], s2 = second[cb];
    int j = bidx[cb];
    if (face >= 0) {
      if (sbox > s1) {
        s2 = fmaxf(s2, s1);
        s1 = sbox;
        j = -2 - face;
      } else {
        s2 = fmaxf(s2, sbox);
      }
    }
    uint8_t st = 0;
    const float thr = fmaxf(a.tau_rel * s1, a.kappa / nn);
    bool tie = !(s1 - s2 > thr);
    float t;
    const int64_t node =
        (j >= 0 && j < n_scan) ? (a.perm ? (int64_t)a.perm[j] : row_node(a, nb0, n_scan, j)) : a.n;
    if (j >= 0 && node >= a.n) {  // cannot happen with the documented MFMA layout; never dereference
      j = -1;
      t = __builtin_nanf("");
      st |= VG_ST_SUSPECT;
      tie = true;
    } else if (j >= 0) {
      j = (int)node;
      t = reeval_cell<DK>(xi, a.nodes + node * d, u, d);
    } else if (j <= -2) {
      t = tbox;
    } else {
      t = __builtin_inff();
      st |= VG_ST_NO_HIT;
      tie = true;
    }
    if constexpr (!GEN) {
      // a non-finite direction read from memory: no answer (drawn ones are finite)
      bool bad = false;
#pragma unroll
      for (int k = 0; k < DK; ++k) bad |= k < d && !__builtin_isfinite(u[k]);
      if (bad) {
        t = __builtin_nanf("");
        j = -1;
        st = VG_ST_BAD_INPUT;
        tie = false;
        atomicAdd(&a.counters[CNT_BAD_RAYS], 1u);
      }
    }
    if (tie && a.flag_list) {
      st |= VG_ST_NEAR_TIE;
      const uint32_t pos = atomicAdd(&a.counters[CNT_FLAGGED], 1u);
      a.flag_list[pos] = gid | a.flag_tag;
    }
    a.t_out[gid] = t;
    a.idx_out[gid] = j;
    a.st_out[gid] = st;
  }
}

// LDS tile of the FP32 scan: row k holds coordinate k of the chunk's NB
// inverted nodes; rows are NB + 32 floats apart so that the two K halves of
// an MFMA operand (lanes 0-31 and 32-63) fall in different bank halves.
template <int KP, int WAVES>
struct Fp32Tile {
  static constexpr int NB = WAVES * 64;
  static constexpr int LS = NB + 32;
  static constexpr int FLOATS = 2 * KP * LS;
};

// Accumulators of one column block of a 32-node block.
template <int KP>
__device__ __forceinline__ f32x16 scan_block(const float (&A)[KP], const float (&ub)[KP]) {
  f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kp = 0; kp < KP; ++kp) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[kp], ub[kp], acc, 0, 0, 0);
  return acc;
}

// One work item of the FP32 scan: rays [chunk*RW, chunk*RW + RW) of `cell`.
// lds holds Fp32Tile<KP, WAVES>::FLOATS floats, NB/32 block bounds,
// 2 x WAVES chunk thresholds and 2 x WAVES window masks, red WAVES*64
// floats, ctab the sorted chunk keys, cen the half-block centres.  One
// accumulator set per wave is reused by the column blocks in turn: separate
// sets would cost the occupancy that hides each block's epilogue.
template <int KP, int C, int WAVES, bool GEN, bool SORTED, bool BIG = false>
__device__ __forceinline__ void scan_fp32_item(const CellScanArgs &a, int64_t cell, int chunk,
                                               float *__restrict__ lds, float *red, float *ctab, float *cen) {
  constexpr int NT = WAVES * 64;
  constexpr int NB = Fp32Tile<KP, WAVES>::NB;  // nodes per LDS chunk (one per thread)
  constexpr int LS = Fp32Tile<KP, WAVES>::LS;
  constexpr int FLOATS = Fp32Tile<KP, WAVES>::FLOATS;
  constexpr int RW = WAVES * C * 32;           // rays per workgroup
  constexpr int DK = 2 * KP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int d = a.d;
  const int64_t n = a.n;
  const int R = a.R;
  if (item_bad_nodes<NT>(a, cell, chunk * RW, RW)) return;

  float xi[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) xi[k] = uniform_f((k < d) ? a.nodes[cell * d + k] : 0.f);

  // B operand: lane l holds u[ray l%32][2kp + l/32] of each column block.
  const int rayw = chunk * RW + wave * (C * 32);
  float ub[C][KP];
#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    const int ray = rayw + cb * 32 + (lane & 31);
    if constexpr (!GEN) {
      const float *up = a.dirs + ((int64_t)cell * R + ray) * d;
#pragma unroll
      for (int kp = 0; kp < KP; ++kp) {
        const int k = 2 * kp + (lane >> 5);
        ub[cb][kp] = (ray < R && k < d) ? up[k] : 0.f;
      }
    } else {
      float u[DK];
      cell_dir<DK>(nullptr, a.seed, cell, R, ray, d, u);
      // component 2kp or 2kp + 1 by a bit mask (a select between the two
      // array elements would become a dynamic index and move u to memory)
      const int hi = (lane & 32) ? -1 : 0;
#pragma unroll
      for (int kp = 0; kp < KP; ++kp)
        ub[cb][kp] = __int_as_float((__float_as_int(u[2 * kp]) & ~hi) | (__float_as_int(u[2 * kp + 1]) & hi));
    }
  }

  // scan order: the skip bounds need |u| = 1 up to rounding for every ray of
  // the workgroup (the two lane halves hold complementary components)
  bool prune = true;
  if constexpr (SORTED) {
    bool unit = true;
#pragma unroll
    for (int cb = 0; cb < C; ++cb) {
      float uu = 0.f;
#pragma unroll
      for (int kp = 0; kp < KP; ++kp) uu = __builtin_fmaf(ub[cb][kp], ub[cb][kp], uu);
      uu += partner32(uu, lane);
      unit = unit && uu <= 1.f + 0x1p-14f;
    }
    prune = __syncthreads_and(unit) != 0;
  }

  float best[C], second[C];
  int bidx[C];
#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    best[cb] = 0.f;  // eligibility: u.r~ > 0
    second[cb] = 0.f;
    bidx[cb] = -1;
  }
  float nn2 = __builtin_inff();

  // A operand: lane l reads row 2kp + l/32, column l%32 of each node block
  const float *lrow = lds + (lane >> 5) * LS + (lane & 31);
  float *bnd = lds + FLOATS;             // NB / 32 block bounds
  float *wsm = lds + FLOATS + NB / 32;   // 2 x WAVES chunk thresholds
  uint32_t *wmask = reinterpret_cast<uint32_t *>(wsm + 2 * WAVES);  // 2 x WAVES window masks
  const int64_t nb0 = a.nbr ? a.nbr_off[cell] : 0;
  const int64_t n_scan = a.nbr ? a.nbr_off[cell + 1] - nb0 : n;
  // block centres (scan order, d >= 3)
  constexpr bool CEN = SORTED && KP >= 2;
  const int blocks = scan_chunks<DK, C, NB, WAVES, SORTED, CEN, SORTED, BIG>(
      a, cell, xi, best, second, nn2, bnd, wsm, wmask, ctab, cen + 16 * 32, nb0, n_scan, rayw, prune,
      [&](const float (&rt)[DK]) {
#pragma unroll
        for (int k = 0; k < DK; ++k) lds[k * LS + tid] = rt[k];
      },
      [&](int nb, int blk16, auto skip) {
        float A[KP];
#pragma unroll
        for (int kp = 0; kp < KP; ++kp) A[kp] = lrow[2 * kp * LS + nb * 32];
        int ran = 0;
#pragma unroll
        for (int cb = 0; cb < C; ++cb) {
          if (skip(cb)) continue;
          const f32x16 acc = scan_block<KP>(A, ub[cb]);
          epilogue16(acc, best[cb], second[cb], bidx[cb], blk16);
          ++ran;
        }
        return ran;
      },
      [&](const float (&c)[DK], int part) {
#pragma unroll
        for (int k = 0; k < DK; ++k) cen[k * 32 + part] = c[k];
      },
      [&](int cb) {
        // u.c for the chunk's half-block centres; the rows past them zero
        constexpr int ROWS = NB / 16;
        float A[KP];
#pragma unroll
        for (int kp = 0; kp < KP; ++kp)
          A[kp] = (lane & 31) < ROWS ? cen[(2 * kp + (lane >> 5)) * 32 + (lane & 31)] : 0.f;
        return scan_block<KP>(A, ub[cb]);
      },
      [&](int cb, const float (&cp)[DK]) {
        // u.c' for the window's 32 inverted ball centres (row l % 32: lane l's)
        const int hi = (lane & 32) ? -1 : 0;
        float A[KP];
#pragma unroll
        for (int kp = 0; kp < KP; ++kp)
          A[kp] = __int_as_float((__float_as_int(cp[2 * kp]) & ~hi) | (__float_as_int(cp[2 * kp + 1]) & hi));
        return scan_block<KP>(A, ub[cb]);
      });

  count_blocks(a, blocks, lane);
  cell_finish<C, DK, NT, GEN>(a, xi, best, second, bidx, nn2, red, lane, rayw, cell, nb0, n_scan);
}

// Workgroup -> (cell, ray chunk).  A launch over a whole cloud in scan order
// takes the cells in the order of the sorted copy (cell perm[p] at position
// p): the workgroups resident at one time then scan nearby cells and share
// the node chunks they load through L2.  Other launches (index order, or a
// probe over the first cells of a cloud) take the cells in index order.
template <bool SORTED>
__device__ __forceinline__ int64_t item_cell(const CellScanArgs &a, int &chunk) {
  const int64_t pos = blockIdx.x / a.wg_per_cell;
  chunk = (int)(blockIdx.x - pos * a.wg_per_cell);
  if (SORTED && (int64_t)gridDim.x == a.n * a.wg_per_cell) return a.perm[pos];
  return pos;
}

// GEN: the directions are drawn from a.seed (a.dirs is null), else read.
// At least two waves per SIMD: with a budget of 256 registers the compiler
// keeps the MFMA accumulators in ordinary VGPRs (with the four-wave shapes it
// would otherwise place them in AGPRs and copy all 16 back per block before
// the epilogue).  The four-wave shapes ask for five (four with four column
// blocks from d = 5 on) and the eight-wave ones up to d = 10 for four: their
// registers then fit without scratch.
// SORTED: the nodes are in scan order (a.xs, a.perm, a.rank, a.aabb).
template <int KP, int C, int WAVES, bool GEN, bool SORTED>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(WAVES == 4 && C == 4 ? (KP <= 2 ? 5 : 4) : (WAVES == 4 && KP <= 6 ? 5 : (WAVES == 8 && KP <= 5 ? 4 : 2))))) void cell_scan_fp32_kernel(
    CellScanArgs a) {
  // tile, NB / 32 block bounds, 2 x WAVES chunk thresholds, 2 x WAVES window masks
  __shared__ float lds[Fp32Tile<KP, WAVES>::FLOATS + WAVES * 2 + WAVES * 2 + WAVES * 2];
  __shared__ float red[WAVES * 64];
  __shared__ float ctab[SORTED ? kChunkTable : 1];  // the walk's chunk keys (chunk_key), sorted
  __shared__ float cen[SORTED ? 16 * 32 + 32 : 1];  // centres [k][part] of (half-)blocks, radii
  int chunk;
  const int64_t cell = item_cell<SORTED>(a, chunk);
  scan_fp32_item<KP, C, WAVES, GEN, SORTED>(a, cell, chunk, lds, red, ctab, cen);
}

// The scan in scan order of a cloud of more chunks than the chunk table
// holds (each table entry shared by consecutive chunks, see scan_chunks).
template <int KP, int C, int WAVES, bool GEN>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(WAVES == 4 && C == 4 ? (KP <= 2 ? 5 : 4) : (WAVES == 4 && KP <= 6 ? 5 : (WAVES == 8 && KP <= 5 ? 4 : 2))))) void cell_scan_fp32_big_kernel(
    CellScanArgs a) {
  __shared__ float lds[Fp32Tile<KP, WAVES>::FLOATS + WAVES * 2 + WAVES * 2 + WAVES * 2];
  __shared__ float red[WAVES * 64];
  __shared__ float ctab[kChunkTable];
  __shared__ float cen[16 * 32 + 32];
  int chunk;
  const int64_t cell = item_cell<true>(a, chunk);
  scan_fp32_item<KP, C, WAVES, GEN, true, true>(a, cell, chunk, lds, red, ctab, cen);
}

// ---------------------------------------------------------------- BF16x3
// Split-precision variant: a = a_hi + a_lo with a_hi = bf16(a) and
// a_lo = bf16(a - a_hi); u.r~ ~ sum hi*hi + hi*lo + lo*hi with FP32
// accumulation.  The three products are packed along K: the node operand is
// [hi | hi | lo] and the direction operand [hi | lo | hi], each block DKP long
// (DKP = 5, 10 or 16 so that 3 DKP fits KQ MFMA K-blocks of 16), padded with
// zeros.  Both operands use the same K slot for the same product, so the
// v_mfma_f32_32x32x16_bf16 K ordering inside a lane does not matter.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KQ>
struct Bf16Pack {
  static constexpr int DKP = KQ == 1 ? 5 : (KQ == 2 ? 10 : 16);
  static constexpr int KT = 16 * KQ;
};

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// Accumulators of one column block of a 32-node block (BF16x3 operands).
template <int KQ>
__device__ __forceinline__ f32x16 scan_block_bf16(const bf16x8 (&A)[KQ], const bf16x8 (&ub)[KQ]) {
  f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < KQ; ++q) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[q], ub[q], acc, 0, 0, 0);
  return acc;
}

// One work item of the BF16x3 scan; lds holds WAVES*64 * KT/8 bf16x8, bnd
// the NB/32 block bounds, 2 x WAVES chunk thresholds and 2 x WAVES window
// masks, ctab the walk's sorted chunk keys.
template <int KQ, int C, int WAVES, bool GEN, bool SORTED, bool BIG = false>
__device__ __forceinline__ void scan_bf16x3_item(const CellScanArgs &a, int64_t cell, int chunk,
                                                 bf16x8 *__restrict__ lds, float *red, float *bnd, float *ctab,
                                                 float *cen) {
  constexpr int NT = WAVES * 64;
  constexpr int NB = NT;
  constexpr int RW = WAVES * C * 32;
  constexpr int DKP = Bf16Pack<KQ>::DKP;
  constexpr int KT = Bf16Pack<KQ>::KT;
  constexpr int DK = DKP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int d = a.d;
  const int64_t n = a.n;
  const int R = a.R;
  if (item_bad_nodes<NT>(a, cell, chunk * RW, RW)) return;

  float xi[DK];
#pragma unroll
  for (int k = 0; k < DK; ++k) xi[k] = uniform_f((k < d) ? a.nodes[cell * d + k] : 0.f);

  const int rayw = chunk * RW + wave * (C * 32);
  bf16x8 ub[C][KQ];
  bool unit = true;  // |u| = 1 up to rounding (the scan-order bounds need it)
#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    const int ray = rayw + cb * 32 + (lane & 31);
    float u[DKP];
    cell_dir<DKP>(GEN ? nullptr : a.dirs, a.seed, cell, R, ray, d, u);
    float uu = 0.f;
#pragma unroll
    for (int k = 0; k < DKP; ++k) uu = __builtin_fmaf(u[k], u[k], uu);
    unit = unit && uu <= 1.f + 0x1p-14f;
    __bf16 uh[DKP], ul[DKP];
#pragma unroll
    for (int k = 0; k < DKP; ++k) split_bf16(u[k], uh[k], ul[k]);
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kk = 16 * q + 8 * h + e;
          v[h] = kk < DKP ? uh[kk % DKP]
                          : (kk < 2 * DKP ? ul[kk % DKP] : (kk < 3 * DKP ? uh[kk % DKP] : (__bf16)0.f));
        }
        ub[cb][q][e] = (lane & 32) ? v[1] : v[0];
      }
    }
  }

  const bool prune = SORTED ? __syncthreads_and(unit) != 0 : true;

  float best[C], second[C];
  int bidx[C];
#pragma unroll
  for (int cb = 0; cb < C; ++cb) {
    best[cb] = 0.f;
    second[cb] = 0.f;
    bidx[cb] = -1;
  }
  float nn2 = __builtin_inff();

  const int64_t nb0 = a.nbr ? a.nbr_off[cell] : 0;
  const int64_t n_scan = a.nbr ? a.nbr_off[cell + 1] - nb0 : n;
  // Half-block centres (as in the FP32 scan) where four column blocks share
  // a chunk's centre work: this scan is VALU-bound and its blocks are cheap,
  // so with fewer rays per wave the per-chunk sums, splits and ballots cost
  // more than the blocks they remove (uniform clouds at 256 rays per cell:
  // 14 to 28 % slower with them; d=10 mixture at 1024 rays: 204 -> 184 ms),
  // and beyond d=10 their registers cost a wave per SIMD.
  constexpr bool CEN = SORTED && C == 4 && KQ <= 2;
  // The window test of the walk: with four column blocks its registers cost
  // a wave per SIMD (3 instead of 4) and the d=10 mixture scan 25 %.
  constexpr bool WIN = SORTED && C <= 2;
  const int blocks = scan_chunks<DK, C, NB, WAVES, SORTED, CEN, WIN, BIG>(
      a, cell, xi, best, second, nn2, bnd, bnd + NB / 32, reinterpret_cast<uint32_t *>(bnd + NB / 32 + 2 * WAVES),
      ctab, cen + 16 * 32, nb0, n_scan, rayw, prune,
      [&](const float (&rt)[DK]) {
        __bf16 rh[DKP], rl[DKP];
#pragma unroll
        for (int k = 0; k < DKP; ++k) split_bf16(rt[k], rh[k], rl[k]);
#pragma unroll
        for (int g = 0; g < KT / 8; ++g) {
          bf16x8 v;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int kk = 8 * g + e;
            v[e] = kk < DKP ? rh[kk % DKP]
                            : (kk < 2 * DKP ? rh[kk % DKP] : (kk < 3 * DKP ? rl[kk % DKP] : (__bf16)0.f));
          }
          lds[tid * (KT / 8) + g] = v;
        }
      },
      [&](int nb, int blk16, auto skip) {
        bf16x8 A[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) A[q] = lds[(nb * 32 + (lane & 31)) * (KT / 8) + 2 * q + (lane >> 5)];
        int ran = 0;
#pragma unroll
        for (int cb = 0; cb < C; ++cb) {
          if (skip(cb)) continue;
          const f32x16 acc = scan_block_bf16<KQ>(A, ub[cb]);
          epilogue16(acc, best[cb], second[cb], bidx[cb], blk16);
          ++ran;
        }
        return ran;
      },
      [&](const float (&c)[DK], int part) {
#pragma unroll
        for (int k = 0; k < DK; ++k) cen[k * 32 + part] = c[k];
      },
      [&](int cb) {
        // u.c for the chunk's half-block centres, split as the nodes; the
        // rows past them zero
        constexpr int ROWS = NB / 16;
        const int row = lane & 31;
        __bf16 ch[DKP], cl[DKP];
#pragma unroll
        for (int k = 0; k < DKP; ++k) split_bf16(row < ROWS ? cen[k * 32 + row] : 0.f, ch[k], cl[k]);
        bf16x8 A[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int kk = 16 * q + 8 * h + e;
              v[h] = kk < DKP ? ch[kk % DKP]
                              : (kk < 2 * DKP ? ch[kk % DKP] : (kk < 3 * DKP ? cl[kk % DKP] : (__bf16)0.f));
            }
            A[q][e] = (lane & 32) ? v[1] : v[0];
          }
        }
        return scan_block_bf16<KQ>(A, ub[cb]);
      },
      [&](int cb, const float (&cp)[DK]) {
        // u.c' for the window's 32 inverted ball centres, split as the nodes
        __bf16 ch[DKP], cl[DKP];
#pragma unroll
        for (int k = 0; k < DKP; ++k) split_bf16(cp[k], ch[k], cl[k]);
        bf16x8 A[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int kk = 16 * q + 8 * h + e;
              v[h] = kk < DKP ? ch[kk % DKP]
                              : (kk < 2 * DKP ? ch[kk % DKP] : (kk < 3 * DKP ? cl[kk % DKP] : (__bf16)0.f));
            }
            A[q][e] = (lane & 32) ? v[1] : v[0];
          }
        }
        return scan_block_bf16<KQ>(A, ub[cb]);
      });
  count_blocks(a, blocks, lane);
  cell_finish<C, DK, NT, GEN>(a, xi, best, second, bidx, nn2, red, lane, rayw, cell, nb0, n_scan);
}

template <int KQ, int C, int WAVES, bool GEN, bool SORTED>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) void cell_scan_bf16x3_kernel(
    CellScanArgs a) {
  __shared__ bf16x8 lds[WAVES * 64 * (Bf16Pack<KQ>::KT / 8)];
  __shared__ float red[WAVES * 64];
  __shared__ float bnd[WAVES * 2 + WAVES * 2 + WAVES * 2];  // block bounds, chunk thresholds, window masks
  __shared__ float ctab[SORTED ? kChunkTable : 1];  // the walk's chunk keys (chunk_key), sorted
  __shared__ float cen[SORTED ? 16 * 32 + 32 : 1];  // half-block centres [k][half], radii
  int chunk;
  const int64_t cell = item_cell<SORTED>(a, chunk);
  scan_bf16x3_item<KQ, C, WAVES, GEN, SORTED>(a, cell, chunk, lds, red, bnd, ctab, cen);
}

// The same for clouds of more chunks than the chunk table holds.
template <int KQ, int C, int WAVES, bool GEN>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) void cell_scan_bf16x3_big_kernel(
    CellScanArgs a) {
  __shared__ bf16x8 lds[WAVES * 64 * (Bf16Pack<KQ>::KT / 8)];
  __shared__ float red[WAVES * 64];
  __shared__ float bnd[WAVES * 2 + WAVES * 2 + WAVES * 2];
  __shared__ float ctab[kChunkTable];
  __shared__ float cen[16 * 32 + 32];
  int chunk;
  const int64_t cell = item_cell<true>(a, chunk);
  scan_bf16x3_item<KQ, C, WAVES, GEN, true, true>(a, cell, chunk, lds, red, bnd, ctab, cen);
}

template <int KQ, int C, int WAVES, bool GEN, bool SORTED, bool BIG>
void launch_kq_one(const CellScanArgs &a, hipStream_t s, int grid) {
  if constexpr (BIG)
    hipLaunchKernelGGL((cell_scan_bf16x3_big_kernel<KQ, C, WAVES, GEN>), dim3(grid), dim3(WAVES * 64), 0, s, a);
  else
    hipLaunchKernelGGL((cell_scan_bf16x3_kernel<KQ, C, WAVES, GEN, SORTED>), dim3(grid), dim3(WAVES * 64), 0, s, a);
}

template <int C, int WAVES, bool GEN, bool SORTED, bool BIG = false>
hipError_t launch_kq_g(const CellScanArgs &a, hipStream_t s, int grid) {
  if (a.d <= 5)
    launch_kq_one<1, C, WAVES, GEN, SORTED, BIG>(a, s, grid);
  else if (a.d <= 10)
    launch_kq_one<2, C, WAVES, GEN, SORTED, BIG>(a, s, grid);
  else
    launch_kq_one<3, C, WAVES, GEN, SORTED, BIG>(a, s, grid);
  return hipGetLastError();
}


template <int C, int WAVES, bool GEN, bool SORTED, bool BIG = false>
hipError_t launch_kp_g(const CellScanArgs &a, hipStream_t s, int grid) {
  const int kp = (a.d + 1) / 2;
  dim3 blk(WAVES * 64);
  switch (kp) {
#define VG_CASE(K)                                                                                        \
  case K:                                                                                                 \
    if constexpr (BIG)                                                                                    \
      hipLaunchKernelGGL((cell_scan_fp32_big_kernel<K, C, WAVES, GEN>), dim3(grid), blk, 0, s, a);        \
    else                                                                                                  \
      hipLaunchKernelGGL((cell_scan_fp32_kernel<K, C, WAVES, GEN, SORTED>), dim3(grid), blk, 0, s, a);    \
    break;
    VG_CASE(1)
    VG_CASE(2)
    VG_CASE(3)
    VG_CASE(4)
    VG_CASE(5)
    VG_CASE(6)
    VG_CASE(7)
    VG_CASE(8)
#undef VG_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 512 rays per workgroup in scan order up to d = 6: four column blocks per
// wave and four waves (256-node chunks) instead of two and eight.  At low d
// a cell needs few chunks: the smaller chunks load fewer nodes the bounds
// rule out, and each chunk's staging and bounds serve 128 rays per wave.
// (Uniform clouds, N = 5e4: d=3 8.4 -> 6.1 ms, d=4 13.2 -> 9.8 ms, d=6
// 38.3 -> 33.1 ms; from d = 8 on, where most chunks run, 2 to 4 % slower.)
// Only while the cloud's 256-node chunks fit the chunk table: beyond it the
// walk goes outward chunk by chunk, and halving the chunks doubles its length
// (d=3, N=4e5, 256 rays in 128-node chunks: 37 -> 328 ms).
template <bool GEN>
hipError_t launch_kp_c4w4(const CellScanArgs &a, hipStream_t s, int grid) {
  dim3 blk(4 * 64);
  switch ((a.d + 1) / 2) {
    case 1: hipLaunchKernelGGL((cell_scan_fp32_kernel<1, 4, 4, GEN, true>), dim3(grid), blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((cell_scan_fp32_kernel<2, 4, 4, GEN, true>), dim3(grid), blk, 0, s, a); break;
    case 3: hipLaunchKernelGGL((cell_scan_fp32_kernel<3, 4, 4, GEN, true>), dim3(grid), blk, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// A cloud in scan order of more chunks (WAVES * 64 nodes each) than the chunk
// table holds takes the big-cloud instance of the shape.
template <int C, int WAVES, bool GEN, bool SORTED>
hipError_t launch_kp_set(const CellScanArgs &a, hipStream_t s, int grid) {
  if constexpr (SORTED)
    if ((a.n + WAVES * 64 - 1) / (WAVES * 64) > kChunkTable) return launch_kp_g<C, WAVES, GEN, true, true>(a, s, grid);
  return launch_kp_g<C, WAVES, GEN, SORTED>(a, s, grid);
}
template <int C, int WAVES, bool GEN, bool SORTED>
hipError_t launch_kq_set(const CellScanArgs &a, hipStream_t s, int grid) {
  if constexpr (SORTED)
    if ((a.n + WAVES * 64 - 1) / (WAVES * 64) > kChunkTable) return launch_kq_g<C, WAVES, GEN, true, true>(a, s, grid);
  return launch_kq_g<C, WAVES, GEN, SORTED>(a, s, grid);
}

// Every tile shape of one (GEN, SORTED) instance set; each set is compiled in
// a translation unit of its own (vg_cell_scan*.hip).
template <bool GEN, bool SORTED>
hipError_t launch_cells_set(const CellScanArgs &a, bool bf16, int rw, int grid, hipStream_t s) {
  if (bf16) {
    switch (rw) {
      case 1024: return launch_kq_set<4, 8, GEN, SORTED>(a, s, grid);
      case 512:
        // d <= 4 in scan order: four column blocks x four waves, as in the
        // FP32 scan (uniform clouds, N = 5e4: d=3 7.2 -> 5.9 ms, d=4 11.6 ->
        // 10.3 ms; from d = 6 on, where four column blocks also turn the
        // centre bound on, -17 to +10 % by cloud, so those keep two x eight)
        if constexpr (SORTED)
          if (a.d <= 4 && a.n <= (int64_t)kChunkTable * 256) {
            launch_kq_one<1, 4, 4, GEN, true, false>(a, s, grid);
            return hipGetLastError();
          }
        return launch_kq_set<2, 8, GEN, SORTED>(a, s, grid);
      case 256: return launch_kq_set<2, 4, GEN, SORTED>(a, s, grid);
      case 128: return launch_kq_set<1, 4, GEN, SORTED>(a, s, grid);
      default: return launch_kq_set<1, 2, GEN, SORTED>(a, s, grid);
    }
  }
  switch (rw) {
    case 1024: return launch_kp_set<4, 8, GEN, SORTED>(a, s, grid);
    case 512:
      if constexpr (SORTED)
        if (a.d <= 6 && a.n <= (int64_t)kChunkTable * 256) return launch_kp_c4w4<GEN>(a, s, grid);
      return launch_kp_set<2, 8, GEN, SORTED>(a, s, grid);
    case 256: return launch_kp_set<2, 4, GEN, SORTED>(a, s, grid);
    case 128: return launch_kp_set<1, 4, GEN, SORTED>(a, s, grid);
    default: return launch_kp_set<1, 2, GEN, SORTED>(a, s, grid);
  }
}

}  // namespace
}  // namespace vg
