// Exhaustive vertex search (Sec. 2.3, Algorithm 2) driven level by level.
//
// Algorithm 2 pops one vertex at a time and casts a ray along each of its
// edges whose visit count G is below 2.  Here a whole breadth-first level is
// popped at once: the edges (vertex, omitted generator) with G < 2 after all
// discoveries of the previous level form one batch of rays, cast on the GPU
// (FP32 scan, FP64 recheck of uncertain rays, no clipping).  New vertices are
// keyed by the sorted (d+1)-tuple sort(eta U {j}); their FP64 coordinates are
// solved on the GPU from the tuple.  The host keeps the vertex set and the
// edge counts in open-addressing hash tables and counts, for every newly
// discovered vertex, each of its d+1 edges (the start vertex included).  A ray
// with no hit is an unbounded edge, recorded as (vertex, omitted generator).
// The vertex set equals the sequential algorithm's: batching only changes the
// order of discovery (and may discover a vertex twice in one level, which the
// set absorbs).
#include <algorithm>
#include <chrono>
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
  int64_t duplicates = 0;
};

using namespace vg;

namespace {

// Open-addressing table from fixed-length int32 tuples to a value.
template <typename V>
class TupleTable {
 public:
  explicit TupleTable(int L) : L_(L) { rehash(1 << 12); }
  size_t size() const { return size_; }
  // Returns the value slot of key, inserting `init` if absent.
  V *find_or_insert(const int32_t *key, V init, bool &inserted) {
    if (2 * (size_ + 1) > cap_) rehash(cap_ * 2);
    size_t s = hash(key) & (cap_ - 1);
    for (;;) {
      if (!used_[s]) {
        used_[s] = 1;
        std::memcpy(&keys_[s * L_], key, sizeof(int32_t) * L_);
        vals_[s] = init;
        ++size_;
        inserted = true;
        return &vals_[s];
      }
      if (!std::memcmp(&keys_[s * L_], key, sizeof(int32_t) * L_)) {
        inserted = false;
        return &vals_[s];
      }
      s = (s + 1) & (cap_ - 1);
    }
  }
  const V *find(const int32_t *key) const {
    size_t s = hash(key) & (cap_ - 1);
    for (;;) {
      if (!used_[s]) return nullptr;
      if (!std::memcmp(&keys_[s * L_], key, sizeof(int32_t) * L_)) return &vals_[s];
      s = (s + 1) & (cap_ - 1);
    }
  }

 private:
  uint64_t hash(const int32_t *k) const {
    uint64_t h = 0x243F6A8885A308D3ull ^ (uint64_t)L_;
    for (int a = 0; a < L_; ++a) {
      h = (h ^ (uint32_t)k[a]) * 0x9E3779B97F4A7C15ull;
      h ^= h >> 29;
    }
    return h ^ (h >> 32);
  }
  void rehash(size_t cap) {
    std::vector<int32_t> ok;
    std::vector<V> ov;
    std::vector<uint8_t> ou;
    ok.swap(keys_);
    ov.swap(vals_);
    ou.swap(used_);
    const size_t ocap = cap_;
    cap_ = cap;
    keys_.assign(cap_ * L_, 0);
    vals_.assign(cap_, V());
    used_.assign(cap_, 0);
    size_ = 0;
    for (size_t s = 0; s < ocap; ++s)
      if (ou[s]) {
        bool ins;
        *find_or_insert(&ok[s * L_], ov[s], ins) = ov[s];
      }
  }
  int L_;
  size_t cap_ = 0, size_ = 0;
  std::vector<int32_t> keys_;
  std::vector<V> vals_;
  std::vector<uint8_t> used_;
};

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

  DevBuf keys_d, coords_d;  // device mirror of the vertex table
  int64_t dev_count = 0;    // vertices mirrored on the device
  DevBuf item_v, item_o, o64, u64, gen, excl, ok, tb, idx, st, nkeys, ncoords, viol;

  bool hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(e);
      return false;
    }
    return true;
  }
};

}  // namespace

extern "C" {

int vg_explore(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, const double *draws,
               int n_draws, uint32_t flags, vg_mesh **out) {
  (void)flags;
  if (!ctx) return VG_EINVAL;
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
  if (n_nodes < d + 1 || n_nodes >= (int64_t(1) << 31) || !nodes || !draws || n_draws < 1) {
    ctx->err = "explore needs n_nodes >= d+1, nodes and descent draws";
    return VG_EINVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ctx->err = "hipSetDevice failed";
    return VG_EDEVICE;
  }
  vg_mesh *M = new (std::nothrow) vg_mesh();
  if (!M) return VG_ENOMEM;
  M->d = d;
  Explorer X{ctx, d, n_nodes, nodes, ctx->stream, {}};
  const int L = d + 1;
  int rc = VG_OK;

#define EX_HIP(call)                        \
  do {                                      \
    if (!X.hip((call), #call)) goto device; \
  } while (0)
#define EX_RC(call)         \
  do {                      \
    rc = (call);            \
    if (rc != VG_OK) goto fail; \
  } while (0)

  {
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
      EX_HIP(hipMemcpyAsync(x0.data(), nodes, sizeof(float) * d, hipMemcpyDeviceToHost, X.s));
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
      EX_HIP(launch_descent_project(nodes, d, sig_d.as<int32_t>(), m, u_d.as<double>(),
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
        EX_RC(raycast_f64(ctx, d, n_nodes, nodes, 1, r_d.as<double>(), u_d.as<double>(),
                          g_d.as<int32_t>(), ex_d.as<int32_t>(), m, 0, true, t32_d.as<float>(),
                          i_d.as<int32_t>(), st_d.as<uint8_t>(), t64_d.as<double>()));
        M->raycasts++;
        EX_HIP(hipMemcpyAsync(&j, i_d.p, sizeof(int32_t), hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipStreamSynchronize(X.s));
      }
      if (j < 0) continue;
      EX_HIP(launch_advance(r_d.as<double>(), u_d.as<double>(), t64_d.as<double>(), d, sign, X.s));
      sig.push_back(j);
    }
    std::sort(sig.begin(), sig.end());
    EX_HIP(hipMemcpyAsync(sig_d.p, sig.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, X.s));
    EX_HIP(launch_solve_one(nodes, d, sig_d.as<int32_t>(), v_d.as<double>(), ok_d.as<int>(), X.s));
    std::vector<double> v0(d);
    int okh = 0;
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
    TupleTable<int64_t> V(L);
    TupleTable<uint8_t> G(d);
    std::vector<int32_t> eta(d);
    auto count_edges = [&](const int32_t *key) {
      for (int o = 0; o <= d; ++o) {
        int q = 0;
        for (int b = 0; b <= d; ++b)
          if (b != o) eta[q++] = key[b];
        bool ins;
        uint8_t *c = G.find_or_insert(eta.data(), 0, ins);
        if (*c < 255) ++*c;
      }
    };
    bool ins;
    *V.find_or_insert(M->sig.data(), 0, ins) = 0;
    count_edges(M->sig.data());
    int64_t level_begin = 0, level_end = 1;
    const bool verbose = std::getenv("VG_VERBOSE") != nullptr;
    const bool validate = std::getenv("VG_VALIDATE") != nullptr;
    const auto t_start = std::chrono::steady_clock::now();
    int level = 0;
    std::vector<int64_t> iv;
    std::vector<int32_t> io, jh, kh;
    std::vector<double> ch;
    while (level_begin < level_end) {
      // frontier: edges of the vertices of this level with G < 2
      iv.clear();
      io.clear();
      for (int64_t v = level_begin; v < level_end; ++v) {
        const int32_t *key = &M->sig[v * L];
        for (int o = 0; o <= d; ++o) {
          int q = 0;
          for (int b = 0; b <= d; ++b)
            if (b != o) eta[q++] = key[b];
          const uint8_t *c = G.find(eta.data());
          if (c && *c >= 2) continue;
          iv.push_back(v);
          io.push_back(o);
        }
      }
      const int64_t m = (int64_t)iv.size();
      // mirror this level's vertices on the device
      const int64_t nv = (int64_t)M->sig.size() / L;
      if (nv > X.dev_count) {
        EX_HIP(X.keys_d.reserve(sizeof(int32_t) * nv * L, true, X.s));
        EX_HIP(X.coords_d.reserve(sizeof(double) * nv * d, true, X.s));
        EX_HIP(hipMemcpyAsync(X.keys_d.as<int32_t>() + X.dev_count * L, &M->sig[X.dev_count * L],
                              sizeof(int32_t) * (nv - X.dev_count) * L, hipMemcpyHostToDevice, X.s));
        EX_HIP(hipMemcpyAsync(X.coords_d.as<double>() + X.dev_count * d,
                              &M->coord[X.dev_count * d],
                              sizeof(double) * (nv - X.dev_count) * d, hipMemcpyHostToDevice, X.s));
        X.dev_count = nv;
      }
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
      EX_HIP(hipMemcpyAsync(X.item_v.p, iv.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, X.s));
      EX_HIP(hipMemcpyAsync(X.item_o.p, io.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, X.s));
      ExploreRays er{};
      er.nodes = nodes;
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
      er.n_nodes = n_nodes;
      EX_HIP(launch_edge_rays(er, X.s));
      EX_RC(raycast_f64(ctx, d, n_nodes, nodes, m, er.o64, er.u64, er.gen, er.excl, d, 0, false,
                        X.tb.as<float>(), X.idx.as<int32_t>(), X.st.as<uint8_t>(), nullptr));
      M->raycasts += m;
      EX_HIP(launch_new_vertices(er, X.s));
      if (validate) {
        // report the edge rays whose new vertex has a node inside its sphere
        EX_HIP(X.viol.reserve(sizeof(double) * m, false, X.s));
        EX_HIP(launch_sphere_check(er, X.viol.as<double>(), X.s));
        std::vector<double> vh(m);
        std::vector<float> th(m);
        std::vector<uint8_t> sh(m);
        EX_HIP(hipMemcpyAsync(vh.data(), X.viol.p, sizeof(double) * m, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipMemcpyAsync(th.data(), X.tb.p, sizeof(float) * m, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipMemcpyAsync(sh.data(), X.st.p, m, hipMemcpyDeviceToHost, X.s));
        std::vector<int32_t> jj(m);
        EX_HIP(hipMemcpyAsync(jj.data(), X.idx.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, X.s));
        EX_HIP(hipStreamSynchronize(X.s));
        int shown = 0;
        int64_t bad = 0;
        for (int64_t it = 0; it < m; ++it) {
          if (vh[it] < -1e-9) {
            ++bad;
            if (shown < 8) {
              ++shown;
              const int32_t *vk = &M->sig[iv[it] * L];
              std::fprintf(stderr, "[explore] level %d item %lld: vertex %lld omit %d hit %d t=%.9g status=%u violation=%.3e coord0=",
                           level + 1, (long long)it, (long long)iv[it], vk[io[it]], jj[it], th[it],
                           (unsigned)sh[it], vh[it]);
              for (int k = 0; k < d; ++k) std::fprintf(stderr, "%.6g ", M->coord[iv[it] * d + k]);
              std::fprintf(stderr, "\n");
            }
          }
        }
        if (bad) {
          std::fprintf(stderr, "[explore] level %d: %lld new vertices violate the empty sphere\n",
                       level + 1, (long long)bad);
          std::fflush(stderr);
          ctx->err = "explore validation failed";
          rc = VG_EINVAL;
          goto fail;
        }
      }
      jh.resize(m);
      kh.resize(m * L);
      ch.resize(m * d);
      EX_HIP(hipMemcpyAsync(jh.data(), X.idx.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipMemcpyAsync(kh.data(), X.nkeys.p, sizeof(int32_t) * m * L, hipMemcpyDeviceToHost, X.s));
      EX_HIP(hipMemcpyAsync(ch.data(), X.ncoords.p, sizeof(double) * m * d, hipMemcpyDeviceToHost,
                            X.s));
      EX_HIP(hipStreamSynchronize(X.s));
      for (int64_t it = 0; it < m; ++it) {
        const int32_t *vkey = &M->sig[iv[it] * L];
        if (jh[it] < 0) {
          M->bsig.insert(M->bsig.end(), vkey, vkey + L);
          M->bomit.push_back(vkey[io[it]]);
          continue;
        }
        const int32_t *nk = &kh[it * L];
        if (nk[0] == -2) {
          ctx->err = "singular vertex (degenerate input)";
          rc = VG_EINVAL;
          goto fail;
        }
        if (nk[0] < 0) continue;
        int64_t *slot = V.find_or_insert(nk, 0, ins);
        if (!ins) {
          M->duplicates++;
          continue;
        }
        *slot = (int64_t)M->sig.size() / L;
        M->sig.insert(M->sig.end(), nk, nk + L);
        M->coord.insert(M->coord.end(), &ch[it * d], &ch[it * d] + d);
        count_edges(nk);
      }
      level_end = (int64_t)M->sig.size() / L;
      ++level;
      if (verbose) {
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        std::fprintf(stderr, "[explore] level %d: %lld rays, %lld new vertices, %lld total, %.2f s\n",
                     level, (long long)m, (long long)(level_end - level_begin),
                     (long long)level_end, el);
        std::fflush(stderr);
      }
    }
  }
  *out = M;
  return VG_OK;

device:
  ctx->err = X.err;
  rc = VG_EDEVICE;
fail:
  delete M;
  return rc;
#undef EX_HIP
#undef EX_RC
}

int64_t vg_mesh_num_vertices(const vg_mesh *m) { return m ? (int64_t)m->sig.size() / (m->d + 1) : -1; }
int64_t vg_mesh_num_unbounded(const vg_mesh *m) { return m ? (int64_t)m->bomit.size() : -1; }
int64_t vg_mesh_num_raycasts(const vg_mesh *m) { return m ? m->raycasts : -1; }

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
