// Device-side bookkeeping of the exhaustive search (Algorithm 2): the set
// of discovered vertices, keyed by sorted (d+1)-tuples of generators, and
// the visit count of every edge, keyed by sorted d-tuples.
//
// Both are open-addressing tables whose slots are claimed with a 64-bit
// compare-and-swap of the key's fingerprint (never 0), so no thread waits on
// another's write.  The full key of a slot is written once, by a single
// owner, and every other user of the slot compares its own key with it in a
// later launch: two different tuples with the same fingerprint are reported
// as a collision, never merged silently.  Probing is linear and bounded by
// the capacity; the host keeps every table at most half full.
//
// Vertex ownership is decided by the smallest global item index (atomicMin),
// so which of several equal new tuples of a level becomes the vertex -- and
// hence the vertex order -- does not depend on scheduling.
#include <hipcub/hipcub.hpp>

#include "vg_explore.h"

namespace vg {
namespace {

constexpr unsigned kBlk = 256;

__device__ __forceinline__ uint64_t tuple_fp(const int32_t *k, int L) {
  uint64_t h = 0x243F6A8885A308D3ull ^ (uint64_t)L;
  for (int a = 0; a < L; ++a) {
    h = (h ^ (uint32_t)k[a]) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
  }
  h ^= h >> 32;
  return h | 1ull;  // 0 marks an empty slot
}

__device__ __forceinline__ bool tuple_eq(const int32_t *a, const int32_t *b, int L) {
  for (int q = 0; q < L; ++q)
    if (a[q] != b[q]) return false;
  return true;
}

// Slot of `fp`, claiming an empty one; -1 when the table is full.
__device__ __forceinline__ int64_t claim(uint64_t *fps, int64_t cap, uint64_t fp) {
  int64_t h = (int64_t)(fp & (uint64_t)(cap - 1));
  for (int64_t probe = 0; probe < cap; ++probe) {
    const unsigned long long old =
        atomicCAS(reinterpret_cast<unsigned long long *>(&fps[h]), 0ull, (unsigned long long)fp);
    if (old == 0ull || old == fp) return h;
    h = (h + 1) & (cap - 1);
  }
  return -1;
}

// Slot holding `fp`, or -1 when absent.
__device__ __forceinline__ int64_t lookup(const uint64_t *fps, int64_t cap, uint64_t fp) {
  int64_t h = (int64_t)(fp & (uint64_t)(cap - 1));
  for (int64_t probe = 0; probe < cap; ++probe) {
    const uint64_t f = fps[h];
    if (f == fp) return h;
    if (f == 0ull) return -1;
    h = (h + 1) & (cap - 1);
  }
  return -1;
}

// The edge of vertex key `key` that omits position o.  On the periodic
// diagram (S > 0) a vertex key's first entry has k = 0; dropping it leaves
// an edge that is translated to the same normal form.  False when that
// fails (shifts outside {-1,0,1}^d).
__device__ __forceinline__ bool edge_of(const int32_t *key, int d, int o, int32_t *eta, int32_t S) {
  int q = 0;
  for (int b = 0; b <= d; ++b)
    if (b != o) eta[q++] = key[b];
  return S == 0 || o != 0 || periodic_canon(eta, d, d, S);
}

__global__ void frontier_flags_kernel(const int32_t *__restrict__ vkeys, int64_t lb, int64_t le,
                                      int d, int32_t face_base, ESet E, uint8_t *__restrict__ flags,
                                      uint32_t *err) {
  const int64_t t = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  const int L = d + 1;
  if (t >= (le - lb) * L) return;
  const int64_t v = lb + t / L;
  const int o = (int)(t - (t / L) * L);
  const int32_t *key = vkeys + v * L;
  // d faces meet in a corner of the cube, not along an edge
  if (key[o] < face_base && (L < 2 || key[1] >= face_base)) {
    flags[t] = 0;
    return;
  }
  int32_t eta[VG_MAX_DIM];
  if (!edge_of(key, d, o, eta, E.S)) {
    atomicOr(err, VSET_RANGE);
    flags[t] = 0;
    return;
  }
  const int64_t h = lookup(E.fp, E.cap, tuple_fp(eta, d));
  uint32_t c = 0;
  if (h >= 0) {
    if (!tuple_eq(E.key + h * d, eta, d)) atomicOr(err, VSET_COLLISION);
    c = E.cnt[h];
  }
  flags[t] = c < 2 ? 1 : 0;
}

__global__ void frontier_items_kernel(const int64_t *__restrict__ sel, int64_t m, int64_t lb, int L,
                                      int64_t *__restrict__ item_v, int32_t *__restrict__ item_o) {
  const int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (p >= m) return;
  const int64_t t = sel[p];
  item_v[p] = lb + t / L;
  item_o[p] = (int32_t)(t - (t / L) * L);
}

// Claim the slot of every new tuple; the smallest global item index owns it.
__global__ void vset_claim_kernel(VSet V, const int32_t *__restrict__ nkeys, const int32_t *__restrict__ idx,
                                  int64_t m, int64_t item_base, int64_t *__restrict__ slot,
                                  uint32_t *err) {
  const int64_t it = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (it >= m) return;
  slot[it] = -1;
  const int32_t *key = nkeys + it * V.L;
  if (idx[it] == -1) return;  // no hit: an unbounded edge (-2-f is a face hit)
  if (key[0] == -2) {
    atomicOr(err, VSET_SINGULAR);
    return;
  }
  if (key[0] < 0) return;
  const int64_t h = claim(V.fp, V.cap, tuple_fp(key, V.L));
  if (h < 0) {
    atomicOr(err, VSET_FULL);
    return;
  }
  atomicMin(reinterpret_cast<long long *>(&V.owner[h]), (long long)(item_base + it));
  slot[it] = h;
}

// Owners write their key; flags mark them (new vertices) and the no-hit items.
__global__ void vset_settle_kernel(VSet V, const int32_t *__restrict__ nkeys, const int32_t *__restrict__ idx,
                                   int64_t m, int64_t item_base, const int64_t *__restrict__ slot,
                                   uint8_t *__restrict__ is_new, uint8_t *__restrict__ is_unb) {
  const int64_t it = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (it >= m) return;
  is_unb[it] = idx[it] == -1 ? 1 : 0;
  const int64_t h = slot[it];
  const bool own = h >= 0 && V.owner[h] == item_base + it;
  is_new[it] = own ? 1 : 0;
  if (own)
    for (int q = 0; q < V.L; ++q) V.key[h * V.L + q] = nkeys[it * V.L + q];
}

// Every other claimant is a duplicate: its key must equal the owner's.
__global__ void vset_verify_kernel(VSet V, const int32_t *__restrict__ nkeys, int64_t m,
                                   const int64_t *__restrict__ slot, const uint8_t *__restrict__ is_new,
                                   uint32_t *err) {
  const int64_t it = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (it >= m) return;
  const int64_t h = slot[it];
  if (h < 0 || is_new[it]) return;
  if (!tuple_eq(V.key + h * V.L, nkeys + it * V.L, V.L)) atomicOr(err, VSET_COLLISION);
}

// Append the new vertices (in item order) and count their edges.
__global__ void append_vertices_kernel(const int64_t *__restrict__ sel, int64_t nn, int64_t nv, int d,
                                       const int32_t *__restrict__ nkeys, const double *__restrict__ ncoords,
                                       int32_t *__restrict__ vkeys, double *__restrict__ vcoords, ESet E,
                                       int64_t *__restrict__ eslot, uint32_t *err) {
  const int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (p >= nn) return;
  const int L = d + 1;
  const int64_t it = sel[p];
  const int32_t *key = nkeys + it * L;
  for (int q = 0; q < L; ++q) vkeys[(nv + p) * L + q] = key[q];
  for (int k = 0; k < d; ++k) vcoords[(nv + p) * d + k] = ncoords[it * d + k];
  int32_t eta[VG_MAX_DIM];
  for (int o = 0; o <= d; ++o) {
    if (!edge_of(key, d, o, eta, E.S)) {
      eslot[p * L + o] = -1;
      atomicOr(err, VSET_RANGE);
      continue;
    }
    const uint64_t fp = tuple_fp(eta, d);
    int64_t h = (int64_t)(fp & (uint64_t)(E.cap - 1));
    int64_t got = -1;
    for (int64_t probe = 0; probe < E.cap; ++probe) {
      const unsigned long long old =
          atomicCAS(reinterpret_cast<unsigned long long *>(&E.fp[h]), 0ull, (unsigned long long)fp);
      if (old == 0ull) {  // first user of the slot writes its key
        for (int q = 0; q < d; ++q) E.key[h * d + q] = eta[q];
        got = h;
        break;
      }
      if (old == fp) {
        got = h;
        break;
      }
      h = (h + 1) & (E.cap - 1);
    }
    eslot[p * L + o] = got;
    if (got < 0) {
      atomicOr(err, VSET_FULL);
      continue;
    }
    atomicAdd(&E.cnt[got], 1u);
  }
}

// Every edge increment's key must equal its slot's key.
__global__ void eset_verify_kernel(const int64_t *__restrict__ sel, int64_t nn, int d,
                                   const int32_t *__restrict__ nkeys, ESet E,
                                   const int64_t *__restrict__ eslot, uint32_t *err) {
  const int64_t t = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  const int L = d + 1;
  if (t >= nn * L) return;
  const int64_t p = t / L;
  const int o = (int)(t - p * L);
  const int64_t h = eslot[t];
  if (h < 0) return;
  int32_t eta[VG_MAX_DIM];
  if (edge_of(nkeys + sel[p] * L, d, o, eta, E.S) && !tuple_eq(E.key + h * d, eta, d))
    atomicOr(err, VSET_COLLISION);
}

__global__ void append_unbounded_kernel(const int64_t *__restrict__ sel, int64_t nb, int64_t b0, int d,
                                        const int64_t *__restrict__ item_v, const int32_t *__restrict__ item_o,
                                        const int32_t *__restrict__ vkeys, int32_t *__restrict__ bsig,
                                        int32_t *__restrict__ bomit) {
  const int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (p >= nb) return;
  const int L = d + 1;
  const int64_t it = sel[p];
  const int32_t *key = vkeys + item_v[it] * L;
  for (int q = 0; q < L; ++q) bsig[(b0 + p) * L + q] = key[q];
  bomit[b0 + p] = key[item_o[it]];
}

// Re-insert vertices [0, nv) into an empty vertex table (owner -1: older
// than every item) and/or count their edges into an empty edge table.
__global__ void rebuild_vset_kernel(VSet V, const int32_t *__restrict__ vkeys, int64_t nv, uint32_t *err) {
  const int64_t v = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (v >= nv) return;
  const int32_t *key = vkeys + v * V.L;
  const int64_t h = claim(V.fp, V.cap, tuple_fp(key, V.L));
  if (h < 0) {
    atomicOr(err, VSET_FULL);
    return;
  }
  V.owner[h] = -1;
  for (int q = 0; q < V.L; ++q) V.key[h * V.L + q] = key[q];
}

__global__ void rebuild_eset_kernel(ESet E, const int32_t *__restrict__ vkeys, int64_t nv, int d,
                                    uint32_t *err) {
  const int64_t v = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (v >= nv) return;
  const int32_t *key = vkeys + v * (d + 1);
  int32_t eta[VG_MAX_DIM];
  for (int o = 0; o <= d; ++o) {
    if (!edge_of(key, d, o, eta, E.S)) {
      atomicOr(err, VSET_RANGE);
      continue;
    }
    const uint64_t fp = tuple_fp(eta, d);
    int64_t h = (int64_t)(fp & (uint64_t)(E.cap - 1));
    int64_t got = -1;
    for (int64_t probe = 0; probe < E.cap; ++probe) {
      const unsigned long long old =
          atomicCAS(reinterpret_cast<unsigned long long *>(&E.fp[h]), 0ull, (unsigned long long)fp);
      if (old == 0ull) {
        for (int q = 0; q < d; ++q) E.key[h * d + q] = eta[q];
        got = h;
        break;
      }
      if (old == fp) {
        got = h;
        break;
      }
      h = (h + 1) & (E.cap - 1);
    }
    if (got < 0) {
      atomicOr(err, VSET_FULL);
      continue;
    }
    atomicAdd(&E.cnt[got], 1u);
  }
}

__global__ void fill_i64_kernel(int64_t *p, int64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  if (i < n) p[i] = v;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlk - 1) / kBlk); }

}  // namespace

hipError_t vset_clear(VSet V, hipStream_t s) {
  hipError_t e = fill_u32(reinterpret_cast<uint32_t *>(V.fp), 0u, 2 * V.cap, s);
  if (e == hipSuccess && V.cap > 0) {
    hipLaunchKernelGGL(fill_i64_kernel, dim3(grid_of(V.cap)), dim3(kBlk), 0, s, V.owner,
                       (int64_t)INT64_MAX, V.cap);
    e = hipGetLastError();
  }
  return e;
}

hipError_t eset_clear(ESet E, hipStream_t s) {
  hipError_t e = fill_u32(reinterpret_cast<uint32_t *>(E.fp), 0u, 2 * E.cap, s);
  if (e == hipSuccess) e = fill_u32(E.cnt, 0u, E.cap, s);
  return e;
}

hipError_t vset_rebuild(VSet V, ESet E, const int32_t *vkeys, int64_t nv, int d, bool vertices,
                        bool edges, uint32_t *err, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  if (vertices) hipLaunchKernelGGL(rebuild_vset_kernel, dim3(grid_of(nv)), dim3(kBlk), 0, s, V, vkeys, nv, err);
  if (edges) hipLaunchKernelGGL(rebuild_eset_kernel, dim3(grid_of(nv)), dim3(kBlk), 0, s, E, vkeys, nv, d, err);
  return hipGetLastError();
}

hipError_t frontier_flags(const int32_t *vkeys, int64_t lb, int64_t le, int d, int32_t face_base, ESet E,
                          uint8_t *flags, uint32_t *err, hipStream_t s) {
  const int64_t cnt = (le - lb) * (d + 1);
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(frontier_flags_kernel, dim3(grid_of(cnt)), dim3(kBlk), 0, s, vkeys, lb, le, d,
                     face_base, E, flags, err);
  return hipGetLastError();
}

hipError_t frontier_items(const int64_t *sel, int64_t m, int64_t lb, int d, int64_t *item_v,
                          int32_t *item_o, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(frontier_items_kernel, dim3(grid_of(m)), dim3(kBlk), 0, s, sel, m, lb, d + 1, item_v,
                     item_o);
  return hipGetLastError();
}

hipError_t vset_insert(VSet V, const int32_t *nkeys, const int32_t *idx, int64_t m, int64_t item_base,
                       int64_t *slot, uint8_t *is_new, uint8_t *is_unb, uint32_t *err, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 g(grid_of(m)), b(kBlk);
  hipLaunchKernelGGL(vset_claim_kernel, g, b, 0, s, V, nkeys, idx, m, item_base, slot, err);
  hipLaunchKernelGGL(vset_settle_kernel, g, b, 0, s, V, nkeys, idx, m, item_base, slot, is_new, is_unb);
  hipLaunchKernelGGL(vset_verify_kernel, g, b, 0, s, V, nkeys, m, slot, is_new, err);
  return hipGetLastError();
}

hipError_t append_vertices(const int64_t *sel, int64_t nn, int64_t nv, int d, const int32_t *nkeys,
                           const double *ncoords, int32_t *vkeys, double *vcoords, ESet E, int64_t *eslot,
                           uint32_t *err, hipStream_t s) {
  if (nn <= 0) return hipSuccess;
  hipLaunchKernelGGL(append_vertices_kernel, dim3(grid_of(nn)), dim3(kBlk), 0, s, sel, nn, nv, d, nkeys,
                     ncoords, vkeys, vcoords, E, eslot, err);
  hipLaunchKernelGGL(eset_verify_kernel, dim3(grid_of(nn * (d + 1))), dim3(kBlk), 0, s, sel, nn, d, nkeys, E,
                     eslot, err);
  return hipGetLastError();
}

hipError_t append_unbounded(const int64_t *sel, int64_t nb, int64_t b0, int d, const int64_t *item_v,
                            const int32_t *item_o, const int32_t *vkeys, int32_t *bsig, int32_t *bomit,
                            hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(append_unbounded_kernel, dim3(grid_of(nb)), dim3(kBlk), 0, s, sel, nb, b0, d, item_v,
                     item_o, vkeys, bsig, bomit);
  return hipGetLastError();
}

// Stable compaction of the indices i < n with flags[i] != 0 (hipCUB); the
// count goes to *count_dev.  Call with temp == nullptr to size temp_bytes.
hipError_t select_flagged(void *temp, size_t &temp_bytes, const uint8_t *flags, int64_t n, int64_t *out,
                          int64_t *count_dev, hipStream_t s) {
  hipcub::CountingInputIterator<int64_t> it(0);
  return hipcub::DeviceSelect::Flagged(temp, temp_bytes, it, flags, out, count_dev, (int)n, s);
}

}  // namespace vg
