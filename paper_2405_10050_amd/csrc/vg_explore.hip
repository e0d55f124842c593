// Exhaustive vertex search (Sec. 2.3, Algorithm 2) driven level by level.
//
// Algorithm 2 pops one vertex at a time and casts a ray along each of its
// edges whose visit count G is below 2.  Here a whole breadth-first level is
// popped at once: the edges (vertex, omitted generator) with G < 2 after all
// discoveries of the previous level form one batch of rays, cast on the GPU
// (FP32 scan, FP64 recheck of uncertain rays, no clipping).  New vertices are
// keyed by the sorted (d+1)-tuple sort(eta U {j}); their FP64 coordinates are
// solved on the GPU from the tuple.  The vertex set and the edge counts are
// device hash tables (vg_vset.hip); every newly discovered vertex counts each
// of its d+1 edges (the start vertex included).  A ray with no hit is an
// unbounded edge, recorded as (vertex, omitted generator).  Frontiers and new
// vertices are compacted in item order, so the vertex order is that of a
// sequential sweep over each level.  The vertex set equals the sequential
// algorithm's: batching only changes the order of discovery (and may
// discover a vertex twice in one level, which the set absorbs).
//
// With VG_CLIP the diagram is clipped to the unit cube: a vertex is fixed by
// d+1 constraints, generators at a common smallest distance and faces x_k = s
// it lies on (key entry n + 2k + s, after the generators).  An edge keeps d
// of them with at least one generator and leaves the vertex away from the
// dropped one; rays are clipped, so a face hit -2-(2k+s) adds that face.
// Every edge is bounded.  The search starts at the corner 0, in the cell of
// its nearest generator, instead of at a Descent.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "vg_explore.h"
#include "vg_internal.h"

struct vg_mesh {
  int d = 0;
  std::vector<int32_t> sig;
  std::vector<double> coord;
  std::vector<int32_t> bsig, bomit;
  int64_t raycasts = 0;
  int64_t nn_calls = 0;  // nearest-neighbour queries of Algorithm 1 (VG_INCIRCLE)
};

using namespace vg;

namespace {

// Device buffer that grows by reallocation (contents not kept unless asked).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t reserve(size_t want, bool keep, hipStream_t s) {
    if (want <= bytes) return hipSuccess;
    size_t nb = std::max(want, bytes * 2);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, nb);
    if (e != hipSuccess) return e;
    if (keep && p && bytes) {
      e = hipMemcpyAsync(q, p, bytes, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        (void)hipFree(q);
        return e;
      }
    }
    if (p) (void)hipFree(p);
    p = q;
    bytes = nb;
    return hipSuccess;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

struct Explorer {
  vg_ctx *ctx;
  int d;
  int64_t n;
  const float *nodes;
  hipStream_t s;
  std::string err;

  DevBuf keys_d, coords_d;                 // vertex list: keys [V][d+1], coordinates [V][d]
  DevBuf vfp, vowner, vkey, efp, ecnt, ekey;  // vertex set and edge counts (VSet, ESet)
  DevBuf bsig_d, bomit_d;                  // unbounded edges
  DevBuf counters, cub, flags, sel, sel2, slot, is_new, is_unb, eslot;
  DevBuf item_v, item_o, o64, u64, gen, excl, ok, tb, idx, st, nkeys, ncoords, viol;

  bool hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(e);
      return false;
    }
    return true;
  }
};

// The scanned images of the periodic search: the images x_i + k,
// k in {-1,0,1}^d, inside [-w, 1+w]^d, as FP32 rows with the k = 0 images
// first (row i is node i), their exact FP64 points, the code of each row and
// the row of each code (-1 outside the layer).
struct ImageLayer {
  int d = 0;
  int32_t S = 0;
  int64_t n = 0;
  const float *nodes = nullptr;          // device
  const std::vector<float> *xh = nullptr;  // host copy of the nodes
  hipStream_t s{};
  double w = 0.0;
  std::vector<int32_t> tkey;
  DevBuf scan, scan64, tkey_d, tix_d;

  // (Re)builds the layer for w_new; a HIP error code or hipSuccess.
  hipError_t build(double w_new) {
    w = w_new;
    const int32_t centre = (S - 1) / 2;
    std::vector<float> rows;
    std::vector<double> rows64;
    std::vector<int32_t> tix((size_t)n * S, -1);
    tkey.clear();
    auto add = [&](int64_t i, int32_t c) {
      double y[VG_MAX_DIM];
      for (int k = 0; k < d; ++k) {
        y[k] = (double)(*xh)[(size_t)i * d + k] + (double)(code_digit(c, k) - 1);
        if (!(y[k] >= -w && y[k] <= 1.0 + w)) return;
      }
      tix[(size_t)i * S + c] = (int32_t)tkey.size();
      tkey.push_back((int32_t)(i * S + c));
      for (int k = 0; k < d; ++k) {
        rows64.push_back(y[k]);
        rows.push_back((float)y[k]);
      }
    };
    for (int64_t i = 0; i < n; ++i) add(i, centre);
    for (int32_t c = 0; c < S; ++c)
      if (c != centre)
        for (int64_t i = 0; i < n; ++i) add(i, c);
    hipError_t e = scan.reserve(sizeof(float) * rows.size(), false, s);
    if (e == hipSuccess) e = scan64.reserve(sizeof(double) * rows64.size(), false, s);
    if (e == hipSuccess) e = tkey_d.reserve(sizeof(int32_t) * tkey.size(), false, s);
    if (e == hipSuccess) e = tix_d.reserve(sizeof(int32_t) * tix.size(), false, s);
    if (e == hipSuccess) e = hipMemcpyAsync(scan.p, rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(scan64.p, rows64.data(), sizeof(double) * rows64.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tkey_d.p, tkey.data(), sizeof(int32_t) * tkey.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tix_d.p, tix.data(), sizeof(int32_t) * tix.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && std::getenv("VG_VERBOSE")) {
      std::fprintf(stderr, "[explore] periodic image layer w = %.4g: %zu rows (%.2f per node)\n", w, tkey.size(),
                   (double)tkey.size() / (double)n);
      std::fflush(stderr);
    }
    return e;
  }
};

// What one search runs over.  Rays are cast over `scan` (n_scan rows): the
// nodes, or on the periodic diagram the images of the scanned layer.
struct Setup {
  int d = 0;
  int64_t n_nodes = 0;
  const float *nodes = nullptr;
  int64_t n_scan = 0;
  const float *scan = nullptr;
  const double *scan64 = nullptr;  // periodic: the exact images the rows were rounded from
  float node_err = 0.f;            // periodic: bound on |row - image|
  const double *draws = nullptr;
  int n_draws = 0;
  bool clipped = false;
  int incircle = 0;
  Periodic per;
  const std::vector<int32_t> *tkey_h = nullptr;  // periodic: code of each scanned image
  const std::vector<float> *xh = nullptr;        // periodic: the nodes, host copy
  ImageLayer *layer = nullptr;                   // periodic: the layer, widened in place

  // Points the scan fields at the layer's current rows.
  void use(const ImageLayer &L) {
    n_scan = (int64_t)L.tkey.size();
    scan = L.scan.as<const float>();
    scan64 = L.scan64.as<const double>();
    // |fl(y) - y| <= 2^-24 |y| per coordinate, |y| <= 1 + w
    node_err = 0x1p-24f * std::sqrt((float)d) * (float)(1.0 + L.w) * 1.01f;
    per.S = L.S;
    per.X = L.nodes;
    per.tkey = L.tkey_d.as<const int32_t>();
    per.tix = L.tix_d.as<const int32_t>();
    per.n_codes = L.n * L.S;
    per.w = L.w;
    tkey_h = &L.tkey;
    xh = L.xh;
  }
};

// One search into M.  On the periodic diagram a level whose new vertex balls
// reach past the image layer is cast again on a layer twice as wide; thin is
// set when that cannot help (w = 1) or the start vertex or an edge key fails.
int explore_run(vg_ctx *ctx, Setup &su, vg_mesh *M, bool &thin) {
  const int d = su.d;
  const int64_t n_nodes = su.n_nodes;
  const float *nodes = su.nodes;
  const bool clipped = su.clipped;
  const int incircle = su.incircle;
  const bool periodic = su.per.S > 0;
  const double *draws = su.draws;
  const int n_draws = su.n_draws;
  Explorer X{ctx, d, su.n_scan, su.scan, ctx->stream, {}};
  const int L = d + 1;
  int rc = VG_OK;
  thin = false;

#define EX_HIP(call)                        \
  do {                                      \
    if (!X.hip((call), #call)) goto device; \
  } while (0)
#define EX_RC(call)         \
  do {                      \
    rc = (call);            \
    if (rc != VG_OK) goto fail; \
  } while (0)

  if (clipped) {
    // ------------------------------------------- start at the corner 0
    std::vector<float> xh((size_t)n_nodes * d);
    EX_HIP(hipMemcpyAsync(xh.data(), nodes, sizeof(float) * xh.size(), hipMemcpyDeviceToHost, X.s));
    EX_HIP(hipStreamSynchronize(X.s));
    int64_t g0 = 0;
    double best = 0.0;
    for (int64_t i = 0; i < n_nodes; ++i) {
      double s2 = 0.0;
      for (int k = 0; k < d; ++k) s2 += (double)xh[i * d + k] * (double)xh[i * d + k];
      if (i == 0 || s2 < best) {
        best = s2;
        g0 = i;
      }
    }
    M->sig.assign(1, (int32_t)g0);
    for (int k = 0; k < d; ++k) M->sig.push_back((int32_t)(n_nodes + 2 * k));
    M->coord.assign(d, 0.0);
  } else {
    // ---------------------------------------------------------- Descent
    // sigma = {0}, r = x_0; each step: next draw, project out span(X_sigma),
    // cast with eta = sigma (FP64 result), r += t u, add the hit generator.
    std::vector<int32_t> sig = {0};
    DevBuf r_d, u_d, sig_d, ok_d, t32_d, i_d, st_d, t64_d, v_d;
    EX_HIP(r_d.reserve(sizeof(double) * d, false, X.s));
    EX_HIP(u_d.reserve(sizeof(double) * d, false, X.s));
    EX_HIP(sig_d.reserve(sizeof(int32_t) * (d + 1), false, X.s));
    EX_HIP(ok_d.reserve(sizeof(int), false, X.s));
    EX_HIP(t32_d.reserve(sizeof(float), false, X.s));
    EX_HIP(i_d.reserve(sizeof(int32_t), false, X.s));
    EX_HIP(st_d.reserve(8, false, X.s));
    EX_HIP(t64_d.reserve(sizeof(double), false, X.s));
    EX_HIP(v_d.reserve(sizeof(double) * d, false, X.s));
    {
      std::vector<float> x0(d);
      EX_HIP(hipMemcpyAsync(x0.data(), su.scan, sizeof(float) * d, hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipStreamSynchronize(X.s));
      std::vector<double> r0(x0.begin(), x0.end());
      EX_HIP(hipMemcpyAsync(r_d.p, r0.data(), sizeof(double) * d, hipMemcpyHostToDevice, X.s));
      EX_HIP(hipStreamSynchronize(X.s));
    }
    int used = 0;
    while ((int)sig.size() < d + 1) {
      if (used >= n_draws) {
        ctx->err = "Descent ran out of random draws";
        rc = VG_EINVAL;
        goto fail;
      }
      EX_HIP(hipMemcpyAsync(u_d.p, draws + (size_t)used * d, sizeof(double) * d,
                            hipMemcpyHostToDevice, X.s));
      ++used;
      const int m = (int)sig.size();
      // the first generator stays first (it is g of eq. (t)); excl is sorted
      EX_HIP(hipMemcpyAsync(sig_d.p, sig.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, X.s));
      EX_HIP(launch_descent_project(su.scan, d, sig_d.as<int32_t>(), m, u_d.as<double>(),
                                    ok_d.as<int>(), X.s));
      int okh = 0;
      EX_HIP(hipMemcpyAsync(&okh, ok_d.p, sizeof(int), hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipStreamSynchronize(X.s));
      if (!okh) continue;
      std::vector<int32_t> ex(sig);
      std::sort(ex.begin(), ex.end());
      DevBuf ex_d, g_d;
      EX_HIP(ex_d.reserve(sizeof(int32_t) * m, false, X.s));
      EX_HIP(g_d.reserve(sizeof(int32_t), false, X.s));
      EX_HIP(hipMemcpyAsync(ex_d.p, ex.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, X.s));
      EX_HIP(hipMemcpyAsync(g_d.p, sig.data(), sizeof(int32_t), hipMemcpyHostToDevice, X.s));
      int32_t j = -1;
      double sign = 1.0;
      for (int attempt = 0; attempt < 2 && j < 0; ++attempt) {
        if (attempt == 1) {
          std::vector<double> uh(d);
          EX_HIP(hipMemcpyAsync(uh.data(), u_d.p, sizeof(double) * d, hipMemcpyDeviceToHost, X.s));
          EX_HIP(hipStreamSynchronize(X.s));
          for (auto &v : uh) v = -v;
          EX_HIP(hipMemcpyAsync(u_d.p, uh.data(), sizeof(double) * d, hipMemcpyHostToDevice, X.s));
          EX_HIP(hipStreamSynchronize(X.s));
        }
        EX_RC(raycast_f64(ctx, d, su.n_scan, su.scan, 1, r_d.as<double>(), u_d.as<double>(),
                          g_d.as<int32_t>(), ex_d.as<int32_t>(), m, 0, true, t32_d.as<float>(),
                          i_d.as<int32_t>(), st_d.as<uint8_t>(), t64_d.as<double>(), incircle, su.scan64,
                          su.node_err));
        M->raycasts++;
        uint64_t calls = 0;
        EX_HIP(hipMemcpyAsync(&j, i_d.p, sizeof(int32_t), hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipMemcpyAsync(&calls, ctx->counters + CNT_NN_CALLS, 8, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipStreamSynchronize(X.s));
        M->nn_calls += (int64_t)calls;
      }
      if (j < 0) continue;
      EX_HIP(launch_advance(r_d.as<double>(), u_d.as<double>(), t64_d.as<double>(), d, sign, X.s));
      sig.push_back(j);
    }
    std::vector<double> v0(d);
    int okh = 0;
    // periodic: rows -> image codes; the ball in the frame of the Descent
    // must lie inside the layer, then the key takes its normal form
    if (periodic)
      for (auto &e : sig) e = (*su.tkey_h)[(size_t)e];
    std::sort(sig.begin(), sig.end());
    if (periodic) {
      EX_HIP(hipMemcpyAsync(sig_d.p, sig.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, X.s));
      EX_HIP(launch_solve_one(su.scan, d, sig_d.as<int32_t>(), su.per, v_d.as<double>(), ok_d.as<int>(), X.s));
      EX_HIP(hipMemcpyAsync(v0.data(), v_d.p, sizeof(double) * d, hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipMemcpyAsync(&okh, ok_d.p, sizeof(int), hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipStreamSynchronize(X.s));
      if (okh) {
        const int32_t i0 = sig[0] / su.per.S, c0 = sig[0] % su.per.S;
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
          const double e = v0[k] - ((double)(*su.xh)[(size_t)i0 * d + k] + (double)(code_digit(c0, k) - 1));
          r2 += e * e;
        }
        const double R = std::sqrt(r2);
        for (int k = 0; k < d; ++k)
          if (!(v0[k] - R > -su.per.w && v0[k] + R < 1.0 + su.per.w)) thin = true;
        if (!periodic_canon(sig.data(), L, d, su.per.S)) thin = true;
        if (thin) {
          ctx->err = "periodic start vertex outside the image layer";
          rc = VG_EUNSUPPORTED;
          goto fail;
        }
      }
    }
    EX_HIP(hipMemcpyAsync(sig_d.p, sig.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, X.s));
    EX_HIP(launch_solve_one(su.scan, d, sig_d.as<int32_t>(), su.per, v_d.as<double>(), ok_d.as<int>(), X.s));
    EX_HIP(hipMemcpyAsync(v0.data(), v_d.p, sizeof(double) * d, hipMemcpyDeviceToHost, X.s));
    EX_HIP(hipMemcpyAsync(&okh, ok_d.p, sizeof(int), hipMemcpyDeviceToHost, X.s));
    EX_HIP(hipStreamSynchronize(X.s));
    if (!okh) {
      ctx->err = "singular start vertex (degenerate input)";
      rc = VG_EINVAL;
      goto fail;
    }
    M->sig.assign(sig.begin(), sig.end());
    M->coord.assign(v0.begin(), v0.end());
  }

  {
    // ------------------------------------------------- breadth-first levels
    // The vertex set, the edge counts, the frontier and the unbounded edges
    // all live on the device; per level the host reads three counts.
    int64_t nv = 1, nb_total = 0, item_base = 0, vcap = 0, ecap = 0;
    const int32_t face_base = clipped ? (int32_t)n_nodes : INT32_MAX;
    uint32_t *errd = nullptr;
    int64_t *cntd = nullptr;
    EX_HIP(X.counters.reserve(64, false, X.s));
    errd = X.counters.as<uint32_t>();
    cntd = reinterpret_cast<int64_t *>(X.counters.as<char>() + 16);
    EX_HIP(fill_u32(errd, 0u, 16, X.s));
    EX_HIP(X.keys_d.reserve(sizeof(int32_t) * L * 1024, false, X.s));
    EX_HIP(X.coords_d.reserve(sizeof(double) * d * 1024, false, X.s));
    EX_HIP(hipMemcpyAsync(X.keys_d.p, M->sig.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, X.s));
    EX_HIP(hipMemcpyAsync(X.coords_d.p, M->coord.data(), sizeof(double) * d, hipMemcpyHostToDevice, X.s));
    // tables at most half full: (re)built from the vertex list when they grow
    auto vset = [&]() {
      return VSet{X.vfp.as<uint64_t>(), X.vowner.as<int64_t>(), X.vkey.as<int32_t>(), vcap, L};
    };
    auto eset = [&]() {
      return ESet{X.efp.as<uint64_t>(), X.ecnt.as<uint32_t>(), X.ekey.as<int32_t>(), ecap, su.per.S};
    };
    auto grow_v = [&](int64_t need) -> hipError_t {
      if (2 * need <= vcap) return hipSuccess;
      int64_t c = int64_t(1) << 16;
      while (c < 4 * need) c <<= 1;
      hipError_t e = X.vfp.reserve(sizeof(uint64_t) * c, false, X.s);
      if (e == hipSuccess) e = X.vowner.reserve(sizeof(int64_t) * c, false, X.s);
      if (e == hipSuccess) e = X.vkey.reserve(sizeof(int32_t) * L * c, false, X.s);
      if (e != hipSuccess) return e;
      vcap = c;
      e = vset_clear(vset(), X.s);
      if (e == hipSuccess) e = vset_rebuild(vset(), eset(), X.keys_d.as<int32_t>(), nv, d, true, false, errd, X.s);
      return e;
    };
    auto grow_e = [&](int64_t need) -> hipError_t {
      if (2 * need <= ecap) return hipSuccess;
      int64_t c = int64_t(1) << 18;
      while (c < 4 * need) c <<= 1;
      hipError_t e = X.efp.reserve(sizeof(uint64_t) * c, false, X.s);
      if (e == hipSuccess) e = X.ecnt.reserve(sizeof(uint32_t) * c, false, X.s);
      if (e == hipSuccess) e = X.ekey.reserve(sizeof(int32_t) * d * c, false, X.s);
      if (e != hipSuccess) return e;
      ecap = c;
      e = eset_clear(eset(), X.s);
      if (e == hipSuccess) e = vset_rebuild(vset(), eset(), X.keys_d.as<int32_t>(), nv, d, false, true, errd, X.s);
      return e;
    };
    // stable compaction of the flagged indices into `out`; returns the count
    auto compact = [&](DevBuf &flags, int64_t n, DevBuf &out, int64_t &count) -> hipError_t {
      size_t tb = 0;
      hipError_t e = select_flagged(nullptr, tb, flags.as<uint8_t>(), n, out.as<int64_t>(), cntd, X.s);
      if (e == hipSuccess) e = X.cub.reserve(std::max<size_t>(tb, 16), false, X.s);
      if (e == hipSuccess) e = select_flagged(X.cub.p, tb, flags.as<uint8_t>(), n, out.as<int64_t>(), cntd, X.s);
      if (e == hipSuccess) e = hipMemcpyAsync(&count, cntd, sizeof(int64_t), hipMemcpyDeviceToHost, X.s);
      if (e == hipSuccess) e = hipStreamSynchronize(X.s);
      return e;
    };
    auto check_err = [&]() -> int {
      uint32_t eh = 0;
      if (hipMemcpyAsync(&eh, errd, sizeof eh, hipMemcpyDeviceToHost, X.s) != hipSuccess ||
          hipStreamSynchronize(X.s) != hipSuccess) {
        ctx->err = "explore: reading the error word failed";
        return VG_EDEVICE;
      }
      if (eh & VSET_SINGULAR) {
        ctx->err = "singular vertex (degenerate input)";
        return VG_EINVAL;
      }
      if (eh & VSET_COLLISION) {
        ctx->err = "explore: two different tuples share a 64-bit fingerprint";
        return VG_EUNSUPPORTED;
      }
      if (eh & VSET_FULL) {
        ctx->err = "explore: a device table ran full";
        return VG_EDEVICE;
      }
      if (eh & (VSET_THIN | VSET_RANGE)) {
        thin = true;
        ctx->err = (eh & VSET_RANGE) ? "periodic key outside the shift range (a vertex ball of radius >= 1/2)"
                                     : "periodic vertex ball past the image layer";
        return VG_EUNSUPPORTED;
      }
      return VG_OK;
    };
    EX_HIP(grow_v(1));
    EX_HIP(grow_e((int64_t)L));
    int64_t level_begin = 0, level_end = 1;
    const bool verbose = std::getenv("VG_VERBOSE") != nullptr;
    const bool validate = std::getenv("VG_VALIDATE") != nullptr && !periodic;
    const auto t_start = std::chrono::steady_clock::now();
    int level = 0;
    while (level_begin < level_end) {
      // frontier: edges of this level's vertices seen fewer than two times
      const int64_t lb = level_begin;
      const int64_t cand = (level_end - level_begin) * L;
      EX_HIP(X.flags.reserve(cand, false, X.s));
      EX_HIP(X.sel.reserve(sizeof(int64_t) * cand, false, X.s));
      EX_HIP(frontier_flags(X.keys_d.as<int32_t>(), level_begin, level_end, d, face_base, eset(),
                            X.flags.as<uint8_t>(), errd, X.s));
      int64_t m = 0;
      EX_HIP(compact(X.flags, cand, X.sel, m));
      EX_RC(check_err());
      level_begin = level_end;
      if (m == 0) break;
      EX_HIP(X.item_v.reserve(sizeof(int64_t) * m, false, X.s));
      EX_HIP(X.item_o.reserve(sizeof(int32_t) * m, false, X.s));
      EX_HIP(X.o64.reserve(sizeof(double) * m * d, false, X.s));
      EX_HIP(X.u64.reserve(sizeof(double) * m * d, false, X.s));
      EX_HIP(X.gen.reserve(sizeof(int32_t) * m, false, X.s));
      EX_HIP(X.excl.reserve(sizeof(int32_t) * m * d, false, X.s));
      EX_HIP(X.ok.reserve(sizeof(int32_t) * m, false, X.s));
      EX_HIP(X.tb.reserve(sizeof(float) * m, false, X.s));
      EX_HIP(X.idx.reserve(sizeof(int32_t) * m, false, X.s));
      EX_HIP(X.st.reserve(m, false, X.s));
      EX_HIP(X.nkeys.reserve(sizeof(int32_t) * m * L, false, X.s));
      EX_HIP(X.ncoords.reserve(sizeof(double) * m * d, false, X.s));
      EX_HIP(X.slot.reserve(sizeof(int64_t) * m, false, X.s));
      EX_HIP(X.is_new.reserve(m, false, X.s));
      EX_HIP(X.is_unb.reserve(m, false, X.s));
      EX_HIP(X.sel2.reserve(sizeof(int64_t) * m, false, X.s));
      EX_HIP(frontier_items(X.sel.as<int64_t>(), m, lb, d, X.item_v.as<int64_t>(), X.item_o.as<int32_t>(),
                            X.s));
      ExploreRays er{};
      er.d = d;
      er.m = m;
      er.keys = X.keys_d.as<int32_t>();
      er.coords = X.coords_d.as<double>();
      er.item_v = X.item_v.as<int64_t>();
      er.item_o = X.item_o.as<int32_t>();
      er.o64 = X.o64.as<double>();
      er.u64 = X.u64.as<double>();
      er.gen = X.gen.as<int32_t>();
      er.excl = X.excl.as<int32_t>();
      er.ok = X.ok.as<int32_t>();
      er.idx = X.idx.as<int32_t>();
      er.new_keys = X.nkeys.as<int32_t>();
      er.new_coords = X.ncoords.as<double>();
      er.face_base = face_base;
      er.err = errd;
      uint32_t flagged = 0;
      for (;;) {
        er.nodes = su.scan;
        er.n_nodes = su.n_scan;
        er.per = su.per;
        EX_HIP(launch_edge_rays(er, X.s));
        EX_RC(raycast_f64(ctx, d, su.n_scan, su.scan, m, er.o64, er.u64, er.gen, er.excl, d, clipped ? 1 : 0, false,
                          X.tb.as<float>(), X.idx.as<int32_t>(), X.st.as<uint8_t>(), nullptr, incircle, su.scan64,
                          su.node_err));
        M->raycasts += m;
        if (verbose) {
          EX_HIP(hipMemcpyAsync(&flagged, ctx->counters + CNT_FLAGGED, 4, hipMemcpyDeviceToHost, X.s));
          EX_HIP(hipStreamSynchronize(X.s));
        }
        if (incircle) {
          uint64_t calls = 0;
          EX_HIP(hipMemcpyAsync(&calls, ctx->counters + CNT_NN_CALLS, 8, hipMemcpyDeviceToHost, X.s));
          EX_HIP(hipStreamSynchronize(X.s));
          M->nn_calls += (int64_t)calls;
        }
        EX_HIP(launch_new_vertices(er, X.s));
        if (!periodic) break;
        // nothing of this level is in the tables yet: if a ball reached past
        // the layer, widen it and cast the level again
        uint32_t eh = 0;
        EX_HIP(hipMemcpyAsync(&eh, errd, sizeof eh, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipStreamSynchronize(X.s));
        if (!(eh & (VSET_THIN | VSET_RANGE)) || su.layer->w >= 1.0) break;
        const uint32_t keep = eh & ~(uint32_t)(VSET_THIN | VSET_RANGE);
        EX_HIP(hipMemcpyAsync(errd, &keep, sizeof keep, hipMemcpyHostToDevice, X.s));
        EX_HIP(su.layer->build(std::min(1.0, 2.0 * su.layer->w)));
        su.use(*su.layer);
        M->raycasts -= m;
      }
      if (validate) {
        // count the edge rays whose new vertex has a node inside its sphere
        EX_HIP(X.viol.reserve(sizeof(double) * m, false, X.s));
        EX_HIP(launch_sphere_check(er, X.viol.as<double>(), X.s));
        std::vector<double> vh(m);
        EX_HIP(hipMemcpyAsync(vh.data(), X.viol.p, sizeof(double) * m, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipStreamSynchronize(X.s));
        int64_t bad = 0, first = -1;
        for (int64_t it = 0; it < m; ++it)
          if (vh[it] < -1e-9 && bad++ == 0) first = it;
        if (bad) {
          std::fprintf(stderr, "[explore] level %d: %lld new vertices violate the empty sphere (first: item %lld, %.3e)\n",
                       level + 1, (long long)bad, (long long)first, vh[first]);
          std::fflush(stderr);
          ctx->err = "explore validation failed";
          rc = VG_EINVAL;
          goto fail;
        }
      }
      // insert the new tuples, then append the new vertices and unbounded edges
      EX_HIP(grow_v(nv + m));
      EX_HIP(vset_insert(vset(), X.nkeys.as<int32_t>(), X.idx.as<int32_t>(), m, item_base, X.slot.as<int64_t>(),
                         X.is_new.as<uint8_t>(), X.is_unb.as<uint8_t>(), errd, X.s));
      int64_t nn = 0, nb = 0;
      EX_HIP(compact(X.is_new, m, X.sel, nn));
      EX_HIP(compact(X.is_unb, m, X.sel2, nb));
      EX_RC(check_err());
      EX_HIP(X.keys_d.reserve(sizeof(int32_t) * L * (nv + nn), true, X.s));
      EX_HIP(X.coords_d.reserve(sizeof(double) * d * (nv + nn), true, X.s));
      EX_HIP(grow_e((int64_t)L * (nv + nn)));
      EX_HIP(X.eslot.reserve(sizeof(int64_t) * L * std::max<int64_t>(nn, 1), false, X.s));
      EX_HIP(append_vertices(X.sel.as<int64_t>(), nn, nv, d, X.nkeys.as<int32_t>(), X.ncoords.as<double>(),
                             X.keys_d.as<int32_t>(), X.coords_d.as<double>(), eset(), X.eslot.as<int64_t>(),
                             errd, X.s));
      if (nb > 0) {
        EX_HIP(X.bsig_d.reserve(sizeof(int32_t) * L * (nb_total + nb), true, X.s));
        EX_HIP(X.bomit_d.reserve(sizeof(int32_t) * (nb_total + nb), true, X.s));
        EX_HIP(append_unbounded(X.sel2.as<int64_t>(), nb, nb_total, d, X.item_v.as<int64_t>(),
                                X.item_o.as<int32_t>(), X.keys_d.as<int32_t>(), X.bsig_d.as<int32_t>(),
                                X.bomit_d.as<int32_t>(), X.s));
      }
      item_base += m;
      nb_total += nb;
      nv += nn;
      level_end = nv;
      ++level;
      if (verbose) {
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        std::fprintf(stderr, "[explore] level %d: %lld rays (%u rechecked), %lld new vertices, %lld total, %.2f s\n",
                     level, (long long)m, flagged, (long long)nn, (long long)nv, el);
        std::fflush(stderr);
      }
    }
    EX_RC(check_err());
    // the mesh is returned in host memory
    M->sig.resize((size_t)nv * L);
    M->coord.resize((size_t)nv * d);
    M->bsig.resize((size_t)nb_total * L);
    M->bomit.resize((size_t)nb_total);
    EX_HIP(hipMemcpyAsync(M->sig.data(), X.keys_d.p, sizeof(int32_t) * L * nv, hipMemcpyDeviceToHost, X.s));
    EX_HIP(hipMemcpyAsync(M->coord.data(), X.coords_d.p, sizeof(double) * d * nv, hipMemcpyDeviceToHost, X.s));
    if (nb_total > 0) {
      EX_HIP(hipMemcpyAsync(M->bsig.data(), X.bsig_d.p, sizeof(int32_t) * L * nb_total, hipMemcpyDeviceToHost,
                            X.s));
      EX_HIP(hipMemcpyAsync(M->bomit.data(), X.bomit_d.p, sizeof(int32_t) * nb_total, hipMemcpyDeviceToHost, X.s));
    }
    EX_HIP(hipStreamSynchronize(X.s));
  }
  return VG_OK;

device:
  ctx->err = X.err;
  rc = VG_EDEVICE;
fail:
  return rc;
#undef EX_HIP
#undef EX_RC
}


}  // namespace

extern "C" {

int vg_explore(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, const double *draws,
               int n_draws, uint32_t flags, vg_mesh **out) {
  if (!ctx) return VG_EINVAL;
  const bool clipped = (flags & VG_CLIP) != 0;
  const bool periodic = (flags & VG_PERIODIC) != 0;
  const int incircle = (flags & VG_INCIRCLE) ? ((flags & VG_INIT_HEURISTIC) ? 2 : 1) : 0;
  ctx->err.clear();
  if (!out) {
    ctx->err = "out is NULL";
    return VG_EINVAL;
  }
  *out = nullptr;
  if (d < 2 || d > VG_MAX_DIM) {
    ctx->err = "d outside [2, VG_MAX_DIM]";
    return VG_EUNSUPPORTED;
  }
  if (flags & ~(uint32_t)(VG_CLIP | VG_INCIRCLE | VG_INIT_HEURISTIC | VG_PERIODIC)) {
    ctx->err = "explore takes VG_CLIP, VG_PERIODIC, VG_INCIRCLE and VG_INIT_HEURISTIC only";
    return VG_EINVAL;
  }
  if (periodic && (clipped || incircle)) {
    ctx->err = "VG_PERIODIC excludes VG_CLIP and VG_INCIRCLE";
    return VG_EUNSUPPORTED;
  }
  if ((flags & VG_INIT_HEURISTIC) && !incircle) {
    ctx->err = "VG_INIT_HEURISTIC needs VG_INCIRCLE";
    return VG_EINVAL;
  }
  if (incircle && d > 6) {
    ctx->err = "VG_INCIRCLE needs d <= 6";
    return VG_EUNSUPPORTED;
  }
  if (clipped ? (n_nodes < 1 || !nodes)
              : ((periodic ? n_nodes < 1 : n_nodes < d + 1) || !nodes || !draws || n_draws < 1)) {
    ctx->err = clipped    ? "clipped explore needs n_nodes >= 1 and nodes"
               : periodic ? "periodic explore needs n_nodes >= 1, nodes and descent draws"
                          : "explore needs n_nodes >= d+1, nodes and descent draws";
    return VG_EINVAL;
  }
  if (n_nodes >= (int64_t(1) << 31) - 2 * VG_MAX_DIM) {
    ctx->err = "n_nodes too large for int32 keys";
    return VG_EINVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ctx->err = "hipSetDevice failed";
    return VG_EDEVICE;
  }
  // non-finite input: the search synchronises anyway, so it is refused here
  std::vector<float> xh((size_t)n_nodes * d);
  if (hipMemcpyAsync(xh.data(), nodes, sizeof(float) * xh.size(), hipMemcpyDeviceToHost, ctx->stream) !=
          hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->err = "copying the nodes failed";
    return VG_EDEVICE;
  }
  for (float x : xh)
    if (!std::isfinite(x)) {
      ctx->err = "non-finite node coordinate";
      return VG_EINVAL;
    }
  if (draws)
    for (int64_t q = 0; q < (int64_t)n_draws * d; ++q)
      if (!std::isfinite(draws[q])) {
        ctx->err = "non-finite descent draw";
        return VG_EINVAL;
      }
  Setup su;
  su.d = d;
  su.n_nodes = n_nodes;
  su.nodes = nodes;
  su.n_scan = n_nodes;
  su.scan = nodes;
  su.draws = draws;
  su.n_draws = n_draws;
  su.clipped = clipped;
  su.incircle = incircle;
  if (!periodic) {
    vg_mesh *M = new (std::nothrow) vg_mesh();
    if (!M) return VG_ENOMEM;
    M->d = d;
    bool thin = false;
    const int rc = explore_run(ctx, su, M, thin);
    if (rc != VG_OK) {
      delete M;
      return rc;
    }
    *out = M;
    return VG_OK;
  }
  // ---------------------------------------------------------- periodic
  // The images x_i + k (k in {-1,0,1}^d) inside [-w, 1+w]^d are scanned;
  // a vertex ball reaching past them (found by the ball check) restarts the
  // search with w doubled, up to w = 1 (every image in [-1,2]^d).
  if (d > 8) {
    ctx->err = "VG_PERIODIC needs d <= 8";
    return VG_EUNSUPPORTED;
  }
  int32_t S = 1;
  for (int a = 0; a < d; ++a) S *= 3;
  if (n_nodes * S >= (int64_t)INT32_MAX) {
    ctx->err = "periodic explore needs n_nodes * 3^d < 2^31 - 1";
    return VG_EUNSUPPORTED;
  }
  for (float x : xh)
    if (!(x >= 0.f && x < 1.f)) {
      ctx->err = "periodic explore needs nodes in [0,1)^d";
      return VG_EINVAL;
    }
  ImageLayer layer;
  layer.d = d;
  layer.S = S;
  layer.n = n_nodes;
  layer.nodes = nodes;
  layer.xh = &xh;
  layer.s = ctx->stream;
  double w = std::min(1.0, 3.0 * std::pow((double)n_nodes, -1.0 / d));
  for (;;) {
    const hipError_t e = layer.build(w);
    if (e != hipSuccess) {
      ctx->err = std::string("periodic image layer: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? VG_ENOMEM : VG_EDEVICE;
    }
    su.use(layer);
    su.layer = &layer;
    vg_mesh *M = new (std::nothrow) vg_mesh();
    if (!M) return VG_ENOMEM;
    M->d = d;
    bool thin = false;
    const int rc = explore_run(ctx, su, M, thin);
    if (rc == VG_OK) {
      *out = M;
      return VG_OK;
    }
    delete M;
    if (!thin) return rc;
    if (layer.w >= 1.0) {
      ctx->err = "periodic explore needs every vertex ball radius below 1/2";
      return VG_EUNSUPPORTED;
    }
    w = std::min(1.0, 2.0 * layer.w);
  }
}

int64_t vg_mesh_num_vertices(const vg_mesh *m) { return m ? (int64_t)m->sig.size() / (m->d + 1) : -1; }
int64_t vg_mesh_num_unbounded(const vg_mesh *m) { return m ? (int64_t)m->bomit.size() : -1; }
int64_t vg_mesh_num_raycasts(const vg_mesh *m) { return m ? m->raycasts : -1; }
int64_t vg_mesh_num_nn_calls(const vg_mesh *m) { return m ? m->nn_calls : -1; }

int vg_mesh_copy(const vg_mesh *m, int32_t *sigma, double *coords, int32_t *b_sigma,
                 int32_t *b_omit) {
  if (!m || !sigma) return VG_EINVAL;
  std::memcpy(sigma, m->sig.data(), sizeof(int32_t) * m->sig.size());
  if (coords) std::memcpy(coords, m->coord.data(), sizeof(double) * m->coord.size());
  if (b_sigma && !m->bsig.empty()) std::memcpy(b_sigma, m->bsig.data(), sizeof(int32_t) * m->bsig.size());
  if (b_omit && !m->bomit.empty()) std::memcpy(b_omit, m->bomit.data(), sizeof(int32_t) * m->bomit.size());
  return VG_OK;
}

void vg_mesh_free(vg_mesh *m) { delete m; }

}  // extern "C"
