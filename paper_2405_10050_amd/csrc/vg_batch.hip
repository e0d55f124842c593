// Uneven batches of RayCast problems in one graph launch.
//
// vg_raycast_cells_batched orders the clouds by decreasing cost (N^2 R
// ceil(d/2): pairs times MFMA K-steps) and captures, once per distinct
// problem table, a hipGraph of: one launch of the single-cloud cell scan per
// cloud -- the exact-K kernel of its dimension, in the tile shape tuned for
// its bucket -- spread over kBranches parallel branches (each cloud goes to
// the branch with the least work so far, largest clouds first), so that the
// clouds' launch tails overlap; then one batched FP64 recheck of the flagged
// rays of every cloud.  Later calls with the same table replay the graph.
// vg_raycast_batched does the same for general rays with one persistent
// kernel over 256-ray tiles of all problems.
//
// Tile shape: the single-cloud scan exists for 64 .. 1024 rays per
// workgroup.  A tuner times, on a probe of each (K-steps, log2 N,
// rays-per-cell, precision) bucket present in a batch -- the first cells of
// that bucket's largest cloud --, half, the default and twice the default
// rays per workgroup for that rays-per-cell, records nanoseconds per
// ray-node pair, and the bucket's clouds use the fastest.  Timings are
// cached in memory and in a text file (VG_TUNE_CACHE, default
// $HOME/.cache/vgraph_tune.txt) so later processes skip the probes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "vg_internal.h"

using namespace vg;

namespace {

constexpr int kBranches = 4;   // parallel branches of a batch graph
constexpr int kNumShapes = 3;  // half, default, twice the default rays per workgroup

struct GraphEntry {
  uint64_t key = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void *table = nullptr;       // BatchProblem[np] on the device
  void *flags = nullptr;       // int64 queue
  void *counters = nullptr;    // CNT_WORDS u32, a u64 item counter at byte 48
  void *status = nullptr;      // status scratch for clouds without status_out
  void *order = nullptr;       // scan-order buffers of the clouds
  int64_t rays = 0;
  uint64_t last_use = 0;
};

struct TuneKey {
  int kp, log2n, R, bf16, ord;  // ord: nodes in scan order
  bool operator<(const TuneKey &o) const {
    return std::tie(kp, log2n, R, bf16, ord) < std::tie(o.kp, o.log2n, o.R, o.bf16, o.ord);
  }
};

struct BatchState {
  hipStream_t capture = nullptr;
  hipStream_t branch[kBranches] = {};
  hipEvent_t fork = nullptr, join[kBranches] = {};
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  std::map<TuneKey, std::vector<double>> tune;  // ns per ray-node pair per shape
  bool tune_loaded = false;
  std::string tune_file;  // the cache file the timings were loaded from
  int cus = 0;
};

void free_entry(GraphEntry &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.table) (void)hipFree(g.table);
  if (g.flags) (void)hipFree(g.flags);
  if (g.counters) (void)hipFree(g.counters);
  if (g.status) (void)hipFree(g.status);
  if (g.order) (void)hipFree(g.order);
  g = GraphEntry{};
}

uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::string tune_path() {
  if (const char *p = std::getenv("VG_TUNE_CACHE")) return p;
  if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/vgraph_tune.txt";
  return "";
}

void load_tune(BatchState &S) {
  S.tune_loaded = true;
  const std::string path = tune_path();
  S.tune_file = path;
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;
  TuneKey k;
  int shape;
  double ns;
  while (std::fscanf(f, "%d %d %d %d %d %d %lf", &k.kp, &k.log2n, &k.R, &k.bf16, &k.ord, &shape, &ns) == 7) {
    if (shape < 0 || shape >= kNumShapes) continue;
    auto &v = S.tune[k];
    v.resize(kNumShapes, -1.0);
    v[shape] = ns;
  }
  std::fclose(f);
}

void save_tune(const BatchState &S) {
  const std::string path = tune_path();
  if (path.empty()) return;
  const std::string tmp = path + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto &kv : S.tune)
    for (int s = 0; s < (int)kv.second.size(); ++s)
      if (kv.second[s] > 0)
        std::fprintf(f, "%d %d %d %d %d %d %.6g\n", kv.first.kp, kv.first.log2n, kv.first.R,
                     kv.first.bf16, kv.first.ord, s, kv.second[s]);
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= n) ++l;
  return l;
}

// Rays per workgroup of shape sh (0: half, 1: the default, 2: twice the
// default for R rays per cell), or 0 when it is outside 64 .. 1024.
int shape_rw(int R, int sh) {
  const int r0 = cell_scan_rays_per_wg(R);
  const int rw = sh == 0 ? r0 / 2 : (sh == 1 ? r0 : 2 * r0);
  return (rw >= 64 && rw <= 1024) ? rw : 0;
}

TuneKey tune_key(const vg_cells_problem &p, bool bf16, uint32_t flags) {
  return TuneKey{(p.d + 1) / 2, ilog2(p.n_nodes), p.rays_per_cell, bf16 ? 1 : 0, scan_order(p.d, flags, bf16) ? 1 : 0};
}

// The scan arguments of one cloud of a batch (q: its position in the table).
CellScanArgs cloud_args(const vg_cells_problem &p, int q, bool bf16, int rw, uint32_t *counters, int64_t *flags,
                        uint8_t *status) {
  CellScanArgs a{};
  a.nodes = p.nodes;
  a.n = p.n_nodes;
  a.d = p.d;
  a.dirs = p.dirs;
  a.R = p.rays_per_cell;
  a.wg_per_cell = (p.rays_per_cell + rw - 1) / rw;
  a.t_out = p.t_out;
  a.idx_out = p.idx_out;
  a.st_out = p.status_out ? p.status_out : status;
  a.counters = counters;
  a.flag_list = flags;
  a.tau_rel = bf16 ? kTauCellsBf16 : kTauCellsFp32;
  a.kappa = cell_kappa(p.d, bf16);
  a.flag_tag = (int64_t)q << 40;
  return a;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the scan-order buffers of one cloud (sort keys, perm, rank, the
// sorted copy and its group boxes and balls), each 256-byte aligned.
size_t order_bytes(const vg_cells_problem &p) {
  const int64_t n = p.n_nodes;
  return align256((size_t)node_order_keys(n) * 8) + 2 * align256((size_t)n * 4) + align256((size_t)(n * p.d) * 4) +
         align256((size_t)order_box_floats(n, p.d) * 4);
}

// Points a's scan-order fields into the buffers at base (order_bytes(p) long).
void carve_order(CellScanArgs &a, const vg_cells_problem &p, char *base, uint64_t *&keys) {
  const int64_t n = p.n_nodes;
  keys = reinterpret_cast<uint64_t *>(base);
  base += align256((size_t)node_order_keys(n) * 8);
  a.perm = reinterpret_cast<int32_t *>(base);
  base += align256((size_t)n * 4);
  a.rank = reinterpret_cast<int32_t *>(base);
  base += align256((size_t)n * 4);
  a.xs = reinterpret_cast<float *>(base);
  base += align256((size_t)(n * p.d) * 4);
  a.aabb = reinterpret_cast<float *>(base);
}

// Device table of a batch (the recheck reads it).  Clouds scanned in scan
// order (scan_order) get their slice of `order` (null: no slices, as for the
// table that only keys the graph cache).
std::vector<BatchProblem> make_table(const std::vector<vg_cells_problem> &pr, const std::vector<int> &order,
                                     const std::vector<int> &rw, bool bf16, uint32_t flags_in, uint32_t *counters,
                                     int64_t *flags, uint8_t *status, char *order_base, int64_t &total_rays,
                                     std::vector<uint64_t *> *keys = nullptr) {
  std::vector<BatchProblem> T(order.size());
  total_rays = 0;
  int64_t status_off = 0;
  size_t order_off = 0;
  if (keys) keys->assign(order.size(), nullptr);
  for (size_t q = 0; q < order.size(); ++q) {
    const vg_cells_problem &p = pr[order[q]];
    const int64_t m = p.n_nodes * (int64_t)p.rays_per_cell;
    T[q].a = cloud_args(p, (int)q, bf16, rw[order[q]], counters, flags,
                        (!p.status_out && status) ? status + status_off : nullptr);
    if (!p.status_out) status_off += m;
    if (order_base && scan_order(p.d, flags_in, bf16)) {
      uint64_t *k = nullptr;
      carve_order(T[q].a, p, order_base + order_off, k);
      if (keys) (*keys)[q] = k;
      order_off += order_bytes(p);
    }
    T[q].item_begin = 0;
    total_rays += m;
  }
  return T;
}

int err(vg_ctx *ctx, int code, const std::string &msg) {
  ctx->err = msg;
  return code;
}

}  // namespace

namespace vg {

void batch_state_free(vg_ctx *ctx) {
  BatchState *S = static_cast<BatchState *>(ctx->batch_state);
  if (!S) return;
  for (auto &g : S->graphs) free_entry(g);
  if (S->capture) (void)hipStreamDestroy(S->capture);
  for (int b = 0; b < kBranches; ++b) {
    if (S->branch[b]) (void)hipStreamDestroy(S->branch[b]);
    if (S->join[b]) (void)hipEventDestroy(S->join[b]);
  }
  if (S->fork) (void)hipEventDestroy(S->fork);
  delete S;
  ctx->batch_state = nullptr;
}

}  // namespace vg

namespace {

BatchState &state(vg_ctx *ctx) {
  if (!ctx->batch_state) ctx->batch_state = new BatchState();
  return *static_cast<BatchState *>(ctx->batch_state);
}

int cus(vg_ctx *ctx) {
  BatchState &S = state(ctx);
  if (!S.cus) {
    hipDeviceProp_t prop;
    S.cus = (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) ? prop.multiProcessorCount : 256;
  }
  return S.cus;
}

// Branch streams and fork/join events of the batch graphs (default priority).
int ensure_branches(vg_ctx *ctx) {
  BatchState &S = state(ctx);
  if (S.fork) return VG_OK;
  for (int b = 0; b < kBranches; ++b)
    if (hipStreamCreateWithFlags(&S.branch[b], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S.join[b], hipEventDisableTiming) != hipSuccess)
      return err(ctx, VG_EDEVICE, "branch stream creation failed");
  if (hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) != hipSuccess)
    return err(ctx, VG_EDEVICE, "branch event creation failed");
  return VG_OK;
}

// Device buffers of one batch: problem table, FP64 recheck queue, counters
// (CNT_WORDS u32, then at byte 48 a u64 item counter), status scratch.
struct BatchBuffers {
  void *table;
  int64_t *flags;
  uint32_t *counters;
  uint8_t *status;
  char *order;  // scan-order buffers of the clouds that use them, or null
};
// Runs the launches of one batch.  The first call with a given key allocates
// the buffers, fills and uploads the table, and captures the launches into a
// hipGraph on a private capture stream; later calls with the same key replay
// that graph on the context's stream (at most 8 graphs are kept, least
// recently used first out).  With VG_NO_GRAPH set, the launches run directly
// and the buffers are freed after a stream synchronisation.
int run_batch(vg_ctx *ctx, uint64_t key, int64_t rays, bool need_status, size_t table_bytes, size_t order_total,
              const std::function<void(const BatchBuffers &, std::vector<char> &)> &fill,
              const std::function<hipError_t(const BatchBuffers &, hipStream_t)> &enqueue,
              float tau) {
  BatchState &S = state(ctx);
  const bool use_graph = std::getenv("VG_NO_GRAPH") == nullptr;
  GraphEntry *g = nullptr;
  for (auto &e : S.graphs)
    if (e.key == key && e.exec) g = &e;
  if (!g || !use_graph) {
    GraphEntry ne;
    ne.key = key;
    ne.rays = rays;
    if (hipMalloc(&ne.flags, (size_t)std::max<int64_t>(rays, 1) * 8) != hipSuccess ||
        hipMalloc(&ne.counters, 64) != hipSuccess ||
        (need_status && hipMalloc(&ne.status, (size_t)std::max<int64_t>(rays, 1)) != hipSuccess) ||
        (order_total && hipMalloc(&ne.order, order_total) != hipSuccess) ||
        hipMalloc(&ne.table, table_bytes) != hipSuccess) {
      free_entry(ne);
      return err(ctx, VG_ENOMEM, "batch buffers allocation failed");
    }
    const BatchBuffers b{ne.table, static_cast<int64_t *>(ne.flags), static_cast<uint32_t *>(ne.counters),
                         static_cast<uint8_t *>(ne.status), static_cast<char *>(ne.order)};
    std::vector<char> bytes;
    fill(b, bytes);
    if (bytes.size() != table_bytes ||
        hipMemcpy(ne.table, bytes.data(), table_bytes, hipMemcpyHostToDevice) != hipSuccess) {
      free_entry(ne);
      return err(ctx, VG_EDEVICE, "batch table upload failed");
    }
    if (!use_graph) {
      hipError_t e = enqueue(b, ctx->stream);
      // keep the buffers alive until the work is done, then drop them
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e == hipSuccess) {
        uint32_t c[CNT_WORDS];
        e = hipMemcpy(c, ne.counters, sizeof c, hipMemcpyDeviceToHost);
        if (e == hipSuccess) (void)hipMemcpy(ctx->counters, c, sizeof c, hipMemcpyHostToDevice);
      }
      free_entry(ne);
      ctx->last_rays = rays;
      ctx->last_tau = tau;
      ctx->last_counters = ctx->counters;
      if (e != hipSuccess) return err(ctx, VG_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
      return VG_OK;
    }
    if (!S.capture && hipStreamCreateWithFlags(&S.capture, hipStreamNonBlocking) != hipSuccess) {
      free_entry(ne);
      return err(ctx, VG_EDEVICE, "capture stream creation failed");
    }
    hipError_t e = hipStreamBeginCapture(S.capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue(b, S.capture);
      e = hipStreamEndCapture(S.capture, &ne.graph);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ne.exec, ne.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      free_entry(ne);
      return err(ctx, VG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (S.graphs.size() >= 8) {
      auto lru = std::min_element(S.graphs.begin(), S.graphs.end(),
                                  [](const GraphEntry &a, const GraphEntry &b) { return a.last_use < b.last_use; });
      (void)hipStreamSynchronize(ctx->stream);
      free_entry(*lru);
      S.graphs.erase(lru);
    }
    S.graphs.push_back(ne);
    g = &S.graphs.back();
  }
  g->last_use = ++S.clock;
  hipError_t e = hipGraphLaunch(g->exec, ctx->stream);
  if (e != hipSuccess) return err(ctx, VG_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  ctx->last_rays = g->rays;
  ctx->last_tau = tau;
  ctx->last_counters = static_cast<uint32_t *>(g->counters);
  return VG_OK;
}

// Time every shape on a probe of each bucket missing from the cache, then
// set rw[i], the rays per workgroup of cloud i, to its bucket's fastest.
int tune(vg_ctx *ctx, const std::vector<vg_cells_problem> &pr, bool bf16, uint32_t call_flags, std::vector<int> &rw) {
  BatchState &S = state(ctx);
  if (!S.tune_loaded || S.tune_file != tune_path()) {
    S.tune.clear();
    load_tune(S);
  }
  std::map<TuneKey, std::vector<int>> buckets;
  for (int i = 0; i < (int)pr.size(); ++i) buckets[tune_key(pr[i], bf16, call_flags)].push_back(i);
  bool changed = false;
  void *counters = nullptr, *flags = nullptr, *ordbuf = nullptr;
  size_t flags_bytes = 0, ord_bytes = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VG_OK;
  for (auto &b : buckets) {
    auto it = S.tune.find(b.first);
    if (it != S.tune.end() && it->second.size() == (size_t)kNumShapes) {
      bool done = true;
      for (int sh = 0; sh < kNumShapes; ++sh)
        done &= it->second[sh] > 0 || !shape_rw(b.first.R, sh);
      if (done) continue;
    }
    if (!counters) {
      if (hipMalloc(&counters, 64) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
          hipEventCreate(&e1) != hipSuccess) {
        rc = err(ctx, VG_EDEVICE, "tuner set-up failed");
        break;
      }
    }
    // probe: the first cells of the bucket's largest cloud
    int big = b.second[0];
    for (int i : b.second)
      if (pr[big].n_nodes < pr[i].n_nodes) big = i;
    const vg_cells_problem &p = pr[big];
    const int64_t cells = std::min<int64_t>(p.n_nodes, 4 * 1024);
    const size_t need = (size_t)(cells * p.rays_per_cell) * 8;
    if (need > flags_bytes) {
      if (flags) (void)hipFree(flags);
      flags = nullptr;
      if (hipMalloc(&flags, need) != hipSuccess) {
        rc = err(ctx, VG_ENOMEM, "tuner queue allocation failed");
        break;
      }
      flags_bytes = need;
    }
    if (!p.status_out) {
      rc = err(ctx, VG_EINVAL, "tuning needs status outputs");
      break;
    }
    // the probe cloud in scan order when its bucket runs that way
    uint64_t *okeys = nullptr;
    CellScanArgs oa{};
    if (b.first.ord) {
      const size_t need_o = order_bytes(p);
      if (need_o > ord_bytes) {
        if (ordbuf) (void)hipFree(ordbuf);
        ordbuf = nullptr;
        if (hipMalloc(&ordbuf, need_o) != hipSuccess) {
          rc = err(ctx, VG_ENOMEM, "tuner order allocation failed");
          break;
        }
        ord_bytes = need_o;
      }
      carve_order(oa, p, static_cast<char *>(ordbuf), okeys);
      if (launch_node_order(p.nodes, p.n_nodes, p.d, okeys, const_cast<int32_t *>(oa.perm),
                            const_cast<int32_t *>(oa.rank), const_cast<float *>(oa.xs), const_cast<float *>(oa.aabb),
                            ctx->stream) != hipSuccess) {
        rc = err(ctx, VG_EDEVICE, "tuner order launch failed");
        break;
      }
    }
    std::vector<double> ns(kNumShapes, -2.0);  // -2: shape not available for this R
    for (int sh = 0; sh < kNumShapes && rc == VG_OK; ++sh) {
      const int r = shape_rw(p.rays_per_cell, sh);
      if (!r) continue;
      CellScanArgs a = cloud_args(p, 0, bf16, r, (uint32_t *)counters, (int64_t *)flags, nullptr);
      a.xs = oa.xs;
      a.perm = oa.perm;
      a.rank = oa.rank;
      a.aabb = oa.aabb;
      // warm-up, then the timed probe
      if (fill_u32((uint32_t *)counters, 0u, 16, ctx->stream) != hipSuccess ||
          launch_cell_scan_rw(a, bf16, r, std::min<int64_t>(cells, 256), ctx->stream) != hipSuccess ||
          fill_u32((uint32_t *)counters, 0u, 16, ctx->stream) != hipSuccess ||
          hipEventRecord(e0, ctx->stream) != hipSuccess ||
          launch_cell_scan_rw(a, bf16, r, cells, ctx->stream) != hipSuccess ||
          hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = err(ctx, VG_EDEVICE, "tuner probe launch failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ns[sh] = ms * 1e6 / ((double)cells * p.rays_per_cell * (double)p.n_nodes);
    }
    if (rc) break;
    S.tune[b.first] = ns;
    changed = true;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (counters) (void)hipFree(counters);
  if (flags) (void)hipFree(flags);
  if (ordbuf) (void)hipFree(ordbuf);
  if (rc) return rc;
  if (changed) save_tune(S);
  for (int i = 0; i < (int)pr.size(); ++i) {
    const auto &v = S.tune[tune_key(pr[i], bf16, call_flags)];
    int best = 1;
    for (int sh = 0; sh < kNumShapes; ++sh)
      if (v[sh] > 0 && shape_rw(pr[i].rays_per_cell, sh) && v[sh] < v[best]) best = sh;
    rw[i] = shape_rw(pr[i].rays_per_cell, best);
  }
  return VG_OK;
}

}  // namespace

extern "C" int vg_raycast_cells_batched(vg_ctx *ctx, int n_problems, const vg_cells_problem *probs,
                                        uint32_t flags) {
  if (!ctx) return VG_EINVAL;
  ctx->err.clear();
  if (n_problems < 0 || (n_problems > 0 && !probs)) return err(ctx, VG_EINVAL, "bad problem table");
  if (n_problems == 0) return VG_OK;
  if (n_problems >= (1 << 22)) return err(ctx, VG_EINVAL, "too many problems");
  if (hipSetDevice(ctx->device) != hipSuccess) return err(ctx, VG_EDEVICE, "hipSetDevice failed");
  const bool bf16 = (flags & VG_PREC_BF16X3) != 0;
  if (flags & VG_NO_RECHECK) return err(ctx, VG_EUNSUPPORTED, "batched calls always recheck");
  if ((flags & VG_SCAN_ORDER) && (flags & VG_INDEX_ORDER))
    return err(ctx, VG_EINVAL, "VG_SCAN_ORDER and VG_INDEX_ORDER exclude each other");
  std::vector<vg_cells_problem> pr(probs, probs + n_problems);
  for (int i = 0; i < n_problems; ++i) {
    const vg_cells_problem &p = pr[i];
    if (p.d < 2 || p.d > VG_MAX_DIM) return err(ctx, VG_EUNSUPPORTED, "problem d outside [2, 16]");
    if (p.n_nodes < 1 || p.n_nodes >= (int64_t(1) << 31))
      return err(ctx, VG_EINVAL, "problem n_nodes outside [1, 2^31)");
    if (p.rays_per_cell < 1 || p.rays_per_cell > 4096)
      return err(ctx, VG_EINVAL, "problem rays_per_cell outside [1, 4096]");
    if (!p.nodes || !p.dirs || !p.t_out || !p.idx_out) return err(ctx, VG_EINVAL, "null problem array");
    if (p.n_nodes * (int64_t)p.rays_per_cell >= (int64_t(1) << 40))
      return err(ctx, VG_EINVAL, "problem too large");
    if (p.n_nodes * ((p.rays_per_cell + 63) / 64) > 0x7fffffff)
      return err(ctx, VG_EINVAL, "problem needs more than 2^31 workgroups");
  }
  int rc = ensure_branches(ctx);
  if (rc) return rc;
  // largest clouds first
  std::vector<int> order(n_problems);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int i) {
    return (double)pr[i].n_nodes * pr[i].n_nodes * pr[i].rays_per_cell * ((pr[i].d + 1) / 2);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<int> rw(n_problems);
  for (int i = 0; i < n_problems; ++i) rw[i] = cell_scan_rays_per_wg(pr[i].rays_per_cell);
  if (const char *e = std::getenv("VG_BATCH_SHAPE")) {
    const int sh = std::max(0, std::min(kNumShapes - 1, std::atoi(e)));
    for (int i = 0; i < n_problems; ++i)
      if (const int r = shape_rw(pr[i].rays_per_cell, sh)) rw[i] = r;
  } else {
    bool have_status = true;
    for (auto &p : pr) have_status &= p.status_out != nullptr;
    if (have_status) {
      rc = tune(ctx, pr, bf16, flags, rw);
      if (rc) return rc;
    }
  }
  // branches: each cloud, largest first, to the branch with the least work
  std::vector<int> branch_of(order.size());
  {
    double load[kBranches] = {};
    for (size_t q = 0; q < order.size(); ++q) {
      const int b = (int)(std::min_element(load, load + kBranches) - load);
      branch_of[q] = b;
      load[b] += cost(order[q]);
    }
  }
  // key: everything the launches depend on
  int64_t rays0;
  std::vector<BatchProblem> probe =
      make_table(pr, order, rw, bf16, flags, nullptr, nullptr, nullptr, nullptr, rays0);
  uint64_t key = fnv(probe.data(), probe.size() * sizeof(BatchProblem));
  key = fnv(&flags, sizeof flags, key);
  bool need_status = false;
  for (auto &p : pr) need_status |= p.status_out == nullptr;
  size_t order_total = 0;
  for (auto &p : pr)
    if (scan_order(p.d, flags, bf16)) order_total += order_bytes(p);
  BatchState &S = state(ctx);
  auto fill = [&](const BatchBuffers &b, std::vector<char> &bytes) {
    int64_t rays;
    std::vector<BatchProblem> T =
        make_table(pr, order, rw, bf16, flags, b.counters, b.flags, b.status, b.order, rays);
    bytes.assign(reinterpret_cast<const char *>(T.data()), reinterpret_cast<const char *>(T.data() + T.size()));
  };
  auto enqueue = [&](const BatchBuffers &b, hipStream_t s) -> hipError_t {
    int64_t rays;
    std::vector<uint64_t *> keys;
    const std::vector<BatchProblem> T =
        make_table(pr, order, rw, bf16, flags, b.counters, b.flags, b.status, b.order, rays, &keys);
    const int rgrid = (int)std::min<int64_t>((rays0 + 3) / 4, 2048);
    hipError_t e = fill_u32(b.counters, 0u, 16, s);
    // fork
    if (e == hipSuccess) e = hipEventRecord(S.fork, s);
    for (int k = 0; k < kBranches && e == hipSuccess; ++k) e = hipStreamWaitEvent(S.branch[k], S.fork, 0);
    for (size_t q = 0; q < T.size() && e == hipSuccess; ++q) {
      const CellScanArgs &a = T[q].a;
      hipStream_t bs = S.branch[branch_of[q]];
      if (a.xs)
        e = launch_node_order(a.nodes, a.n, a.d, keys[q], const_cast<int32_t *>(a.perm),
                              const_cast<int32_t *>(a.rank), const_cast<float *>(a.xs), const_cast<float *>(a.aabb),
                              bs);
      if (e == hipSuccess) e = launch_cell_scan_rw(a, bf16, rw[order[q]], a.n, bs);
    }
    // join
    for (int k = 0; k < kBranches && e == hipSuccess; ++k) {
      e = hipEventRecord(S.join[k], S.branch[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, S.join[k], 0);
    }
    if (e == hipSuccess)
      e = launch_recheck_batched((const BatchProblem *)b.table, b.counters, b.flags, b.counters + CNT_FP64_TIE,
                                 std::max(rgrid, 1), s);
    return e;
  };
  return run_batch(ctx, key, rays0, need_status, probe.size() * sizeof(BatchProblem), order_total, fill, enqueue,
                   bf16 ? kTauCellsBf16 : kTauCellsFp32);
}


// Problems with rays, largest first (n_rays * n_nodes * d), as a device
// table; items are 256-ray tiles.
static std::vector<RayBatchProblem> make_rays_table(const std::vector<vg_rays_problem> &pr,
                                                    const std::vector<int> &order, int clip,
                                                    uint32_t *counters, int64_t *flags,
                                                    uint8_t *status, int64_t &total_items,
                                                    int64_t &total_rays) {
  std::vector<RayBatchProblem> T(order.size());
  total_items = 0;
  total_rays = 0;
  int64_t status_off = 0;
  for (size_t q = 0; q < order.size(); ++q) {
    const vg_rays_problem &p = pr[order[q]];
    RayScanArgs &a = T[q].a;
    a = RayScanArgs{};
    a.nodes = p.nodes;
    a.n = p.n_nodes;
    a.d = p.d;
    a.m = p.n_rays;
    a.o32 = p.origin;
    a.u32 = p.dir;
    a.gen = p.gen;
    a.excl = p.n_excl > 0 ? p.excl : nullptr;
    a.n_excl = p.n_excl;
    a.clip = clip;
    a.t_out = p.t_out;
    a.idx_out = p.idx_out;
    if (p.status_out) {
      a.st_out = p.status_out;
    } else {
      a.st_out = status ? status + status_off : nullptr;
      status_off += p.n_rays;
    }
    a.counters = counters;
    a.flag_list = flags;
    a.tau = kTauRays;
    a.flag_tag = (int64_t)q << 40;
    T[q].item_begin = total_items;
    total_items += (p.n_rays + kRayTile - 1) / kRayTile;
    total_rays += p.n_rays;
  }
  return T;
}

extern "C" int vg_raycast_batched(vg_ctx *ctx, int n_problems, const vg_rays_problem *probs,
                                  uint32_t flags) {
  if (!ctx) return VG_EINVAL;
  ctx->err.clear();
  if (n_problems < 0 || (n_problems > 0 && !probs)) return err(ctx, VG_EINVAL, "bad problem table");
  if (n_problems >= (1 << 22)) return err(ctx, VG_EINVAL, "too many problems");
  if (flags & VG_NO_RECHECK) return err(ctx, VG_EUNSUPPORTED, "batched calls always recheck");
  if (flags & VG_PREC_BF16X3) return err(ctx, VG_EUNSUPPORTED, "general rays scan in FP32 only");
  std::vector<vg_rays_problem> pr(probs, probs + n_problems);
  std::vector<int> order;
  for (int i = 0; i < n_problems; ++i) {
    const vg_rays_problem &p = pr[i];
    if (p.d < 2 || p.d > VG_MAX_DIM) return err(ctx, VG_EUNSUPPORTED, "problem d outside [2, 16]");
    if (p.n_nodes < 1 || p.n_nodes >= (int64_t(1) << 31))
      return err(ctx, VG_EINVAL, "problem n_nodes outside [1, 2^31)");
    if (!p.nodes) return err(ctx, VG_EINVAL, "null problem nodes");
    if (p.n_rays < 0 || p.n_rays >= (int64_t(1) << 40))
      return err(ctx, VG_EINVAL, "problem n_rays outside [0, 2^40)");
    if (p.n_excl < 0 || p.n_excl > p.d) return err(ctx, VG_EINVAL, "problem n_excl outside [0, d]");
    if (p.n_rays == 0) continue;
    if (!p.origin || !p.dir || !p.gen || !p.t_out || !p.idx_out)
      return err(ctx, VG_EINVAL, "null problem ray array");
    if (p.n_excl > 0 && !p.excl) return err(ctx, VG_EINVAL, "problem excl is NULL with n_excl > 0");
    order.push_back(i);
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return err(ctx, VG_EDEVICE, "hipSetDevice failed");
  if (order.empty()) {
    ctx->last_rays = 0;
    return VG_OK;
  }
  auto cost = [&](int i) { return (double)pr[i].n_rays * (double)pr[i].n_nodes * pr[i].d; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  const int clip = (flags & VG_CLIP) ? 1 : 0;
  const int np = (int)order.size();

  int64_t items0, rays0;
  std::vector<RayBatchProblem> probe =
      make_rays_table(pr, order, clip, nullptr, nullptr, nullptr, items0, rays0);
  static const char tag[] = "general rays";
  uint64_t key = fnv(tag, sizeof tag);
  key = fnv(probe.data(), probe.size() * sizeof(RayBatchProblem), key);
  key = fnv(&flags, sizeof flags, key);
  bool need_status = false;
  for (int i : order) need_status |= pr[i].status_out == nullptr;
  BatchState &S = state(ctx);
  if (!S.cus) {
    hipDeviceProp_t prop;
    S.cus = (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) ? prop.multiProcessorCount : 256;
  }
  const int grid = (int)std::min<int64_t>(items0, (int64_t)S.cus * ray_scan_batched_blocks_per_cu());
  auto fill = [&](const BatchBuffers &b, std::vector<char> &bytes) {
    int64_t items, rays;
    std::vector<RayBatchProblem> T =
        make_rays_table(pr, order, clip, b.counters, b.flags, b.status, items, rays);
    bytes.assign(reinterpret_cast<const char *>(T.data()),
                 reinterpret_cast<const char *>(T.data() + T.size()));
  };
  auto enqueue = [&](const BatchBuffers &b, hipStream_t s) -> hipError_t {
    const int rgrid = (int)std::min<int64_t>((rays0 + 3) / 4, 2048);
    unsigned long long *next = reinterpret_cast<unsigned long long *>((char *)b.counters + 48);
    hipError_t e = fill_u32(b.counters, 0u, 16, s);
    if (e == hipSuccess)
      e = launch_ray_scan_batched((const RayBatchProblem *)b.table, np, items0, next, grid, s);
    if (e == hipSuccess)
      e = launch_recheck_rays_batched((const RayBatchProblem *)b.table, b.counters, b.flags,
                                      b.counters + CNT_FP64_TIE, std::max(rgrid, 1), s);
    return e;
  };
  return run_batch(ctx, key, rays0, need_status, probe.size() * sizeof(RayBatchProblem), 0, fill,
                   enqueue, kTauRays);
}
