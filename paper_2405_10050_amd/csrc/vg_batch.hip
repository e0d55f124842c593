// Uneven batches of RayCast problems in persistent launches.
//
// vg_raycast_cells_batched groups the clouds by register class of their K
// extent (one persistent kernel per class keeps the occupancy of the small
// extents), orders them by decreasing cost within a class (N^2 R ceil(d/2):
// pairs times MFMA K-steps), lays their (cell, ray-chunk) items out in that
// order, and runs per class one persistent scan kernel that takes items from
// a device counter; then one batched FP64 recheck.  vg_raycast_batched does
// the same for general rays (one persistent kernel over 256-ray tiles of all
// problems).  The launches (counter fill, scans, recheck) are captured once
// into a hipGraph per distinct problem table and replayed on later calls with
// the same table.
//
// Tile shape: the persistent cell kernels exist in a few shapes (rays per
// item, waves per workgroup).  A tuner times every shape on a probe of each
// (K-steps, log2 N, rays-per-cell, precision) bucket present in a batch --
// the first items of that bucket's clouds -- records nanoseconds per
// ray-node pair, and picks the shape with the smallest predicted batch time.
// Timings are cached in memory and in a text file (VG_TUNE_CACHE, default
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

struct GraphEntry {
  uint64_t key = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void *table = nullptr;       // BatchProblem[np] on the device
  void *flags = nullptr;       // int64 queue
  void *counters = nullptr;    // CNT_WORDS u32 + u64 item counter
  void *status = nullptr;      // status scratch for clouds without status_out
  int64_t rays = 0;
  uint64_t last_use = 0;
};

struct TuneKey {
  int kp, log2n, R, bf16;
  bool operator<(const TuneKey &o) const {
    return std::tie(kp, log2n, R, bf16) < std::tie(o.kp, o.log2n, o.R, o.bf16);
  }
};

struct BatchState {
  hipStream_t capture = nullptr;
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  std::map<TuneKey, std::vector<double>> tune;  // ns per ray-node pair per shape
  bool tune_loaded = false;
  int cus = 0;
};

void free_entry(GraphEntry &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.table) (void)hipFree(g.table);
  if (g.flags) (void)hipFree(g.flags);
  if (g.counters) (void)hipFree(g.counters);
  if (g.status) (void)hipFree(g.status);
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
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;
  TuneKey k;
  int shape;
  double ns;
  while (std::fscanf(f, "%d %d %d %d %d %lf", &k.kp, &k.log2n, &k.R, &k.bf16, &shape, &ns) == 6) {
    if (shape < 0 || shape >= kNumBatchShapes) continue;
    auto &v = S.tune[k];
    v.resize(kNumBatchShapes, -1.0);
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
        std::fprintf(f, "%d %d %d %d %d %.6g\n", kv.first.kp, kv.first.log2n, kv.first.R,
                     kv.first.bf16, s, kv.second[s]);
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

int rays_per_item(int shape) { return 32 * kBatchShapes[shape].C * kBatchShapes[shape].waves; }

int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= n) ++l;
  return l;
}

// Device table of a batch for a given shape (host side).
std::vector<BatchProblem> make_table(const std::vector<vg_cells_problem> &pr,
                                     const std::vector<int> &order, int shape, bool bf16,
                                     uint32_t *counters, int64_t *flags, uint8_t *status,
                                     int64_t &total_items, int64_t &total_rays) {
  std::vector<BatchProblem> T(order.size());
  const int rw = rays_per_item(shape);
  total_items = 0;
  total_rays = 0;
  int64_t status_off = 0;
  for (size_t q = 0; q < order.size(); ++q) {
    const vg_cells_problem &p = pr[order[q]];
    CellScanArgs &a = T[q].a;
    a = CellScanArgs{};
    a.nodes = p.nodes;
    a.n = p.n_nodes;
    a.d = p.d;
    a.dirs = p.dirs;
    a.R = p.rays_per_cell;
    a.wg_per_cell = (p.rays_per_cell + rw - 1) / rw;
    a.t_out = p.t_out;
    a.idx_out = p.idx_out;
    const int64_t m = p.n_nodes * (int64_t)p.rays_per_cell;
    if (p.status_out) {
      a.st_out = p.status_out;
    } else {
      a.st_out = status ? status + status_off : nullptr;
      status_off += m;
    }
    a.counters = counters;
    a.flag_list = flags;
    a.tau_rel = bf16 ? kTauCellsBf16 : kTauCellsFp32;
    a.kappa = cell_kappa(p.d, bf16);
    a.flag_tag = (int64_t)q << 40;
    T[q].item_begin = total_items;
    total_items += p.n_nodes * a.wg_per_cell;
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
  delete S;
  ctx->batch_state = nullptr;
}

}  // namespace vg

namespace {

BatchState &state(vg_ctx *ctx) {
  if (!ctx->batch_state) ctx->batch_state = new BatchState();
  return *static_cast<BatchState *>(ctx->batch_state);
}

int persistent_grid(vg_ctx *ctx, int shape, bool bf16, int cls) {
  BatchState &S = state(ctx);
  if (!S.cus) {
    hipDeviceProp_t prop;
    S.cus = (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) ? prop.multiProcessorCount : 256;
  }
  return S.cus * batched_blocks_per_cu(shape, bf16, cls);
}

// Device buffers of one batch: problem table, FP64 recheck queue, counters
// (CNT_WORDS u32, then from byte 32 one u64 item counter per launch, at most
// four), status scratch.
struct BatchBuffers {
  void *table;
  int64_t *flags;
  uint32_t *counters;
  uint8_t *status;
};

// Runs the launches of one batch.  The first call with a given key allocates
// the buffers, fills and uploads the table, and captures the launches into a
// hipGraph on a private capture stream; later calls with the same key replay
// that graph on the context's stream (at most 8 graphs are kept, least
// recently used first out).  With VG_NO_GRAPH set, the launches run directly
// and the buffers are freed after a stream synchronisation.
int run_batch(vg_ctx *ctx, uint64_t key, int64_t rays, bool need_status, size_t table_bytes,
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
        hipMalloc(&ne.table, table_bytes) != hipSuccess) {
      free_entry(ne);
      return err(ctx, VG_ENOMEM, "batch buffers allocation failed");
    }
    const BatchBuffers b{ne.table, static_cast<int64_t *>(ne.flags), static_cast<uint32_t *>(ne.counters),
                         static_cast<uint8_t *>(ne.status)};
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

// Time every shape on a probe of each bucket missing from the cache.
int tune(vg_ctx *ctx, const std::vector<vg_cells_problem> &pr, bool bf16) {
  BatchState &S = state(ctx);
  if (!S.tune_loaded) load_tune(S);
  std::map<TuneKey, std::vector<int>> buckets;
  for (int i = 0; i < (int)pr.size(); ++i)
    buckets[{(pr[i].d + 1) / 2, ilog2(pr[i].n_nodes), pr[i].rays_per_cell, bf16 ? 1 : 0}].push_back(i);
  bool changed = false;
  void *counters = nullptr, *flags = nullptr, *tab = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VG_OK;
  for (auto &b : buckets) {
    auto it = S.tune.find(b.first);
    if (it != S.tune.end() && std::all_of(it->second.begin(), it->second.end(),
                                          [](double v) { return v > 0; }))
      continue;
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
      if (pr[i].n_nodes > pr[big].n_nodes) big = i;
    std::vector<double> ns(kNumBatchShapes, -1.0);
    for (int sh = 0; sh < kNumBatchShapes; ++sh) {
      const int64_t cells = std::min<int64_t>(pr[big].n_nodes, 4 * 1024);
      std::vector<int> one = {big};
      int64_t items, rays;
      const int64_t m = pr[big].n_nodes * (int64_t)pr[big].rays_per_cell;
      if (flags) (void)hipFree(flags);
      flags = nullptr;
      if (hipMalloc(&flags, (size_t)m * 8) != hipSuccess) {
        rc = err(ctx, VG_ENOMEM, "tuner queue allocation failed");
        break;
      }
      std::vector<BatchProblem> T =
          make_table(pr, one, sh, bf16, (uint32_t *)counters, (int64_t *)flags,
                     nullptr, items, rays);
      if (!pr[big].status_out) {
        rc = err(ctx, VG_EINVAL, "tuning needs status outputs");
        break;
      }
      if (!tab && hipMalloc(&tab, sizeof(BatchProblem)) != hipSuccess) {
        rc = err(ctx, VG_ENOMEM, "tuner table allocation failed");
        break;
      }
      const int64_t probe_items = std::min<int64_t>(items, cells * T[0].a.wg_per_cell);
      if (hipMemcpyAsync(tab, T.data(), sizeof(BatchProblem), hipMemcpyHostToDevice, ctx->stream) !=
              hipSuccess ||
          fill_u32((uint32_t *)counters, 0u, 16, ctx->stream) != hipSuccess) {
        rc = err(ctx, VG_EDEVICE, "tuner upload failed");
        break;
      }
      const int cls = batched_class(pr[big].d, bf16);
      const int grid = persistent_grid(ctx, sh, bf16, cls);
      unsigned long long *next = reinterpret_cast<unsigned long long *>((char *)counters + 32);
      // warm-up, then timed run of the probe
      if (launch_cell_scan_batched((const BatchProblem *)tab, 1, 0, std::min<int64_t>(probe_items, grid),
                                   next, sh, bf16, cls, grid, ctx->stream) != hipSuccess ||
          fill_u32((uint32_t *)counters, 0u, 16, ctx->stream) != hipSuccess ||
          hipEventRecord(e0, ctx->stream) != hipSuccess ||
          launch_cell_scan_batched((const BatchProblem *)tab, 1, 0, probe_items, next, sh, bf16, cls, grid,
                                   ctx->stream) != hipSuccess ||
          hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = err(ctx, VG_EDEVICE, "tuner probe launch failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double pairs = (double)probe_items / T[0].a.wg_per_cell * pr[big].rays_per_cell *
                           (double)pr[big].n_nodes;
      ns[sh] = ms * 1e6 / pairs;
    }
    if (rc) break;
    S.tune[b.first] = ns;
    changed = true;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (counters) (void)hipFree(counters);
  if (flags) (void)hipFree(flags);
  if (tab) (void)hipFree(tab);
  if (rc) return -1;
  if (changed) save_tune(S);
  // predicted batch time per shape
  int best = 0;
  double best_t = 1e300;
  for (int sh = 0; sh < kNumBatchShapes; ++sh) {
    double t = 0;
    for (auto &p : pr) {
      const auto &v = S.tune[{(p.d + 1) / 2, ilog2(p.n_nodes), p.rays_per_cell, bf16 ? 1 : 0}];
      t += v[sh] * (double)p.n_nodes * p.rays_per_cell * (double)p.n_nodes;
    }
    if (t < best_t) {
      best_t = t;
      best = sh;
    }
  }
  return best;
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
  }
  // grouped by register class, largest clouds first within a class
  std::vector<int> order(n_problems);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int i) {
    return (double)pr[i].n_nodes * pr[i].n_nodes * pr[i].rays_per_cell * ((pr[i].d + 1) / 2);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ca = batched_class(pr[a].d, bf16), cb = batched_class(pr[b].d, bf16);
    return ca != cb ? ca < cb : cost(a) > cost(b);
  });

  int shape = 0;
  if (const char *e = std::getenv("VG_BATCH_SHAPE")) {
    shape = std::max(0, std::min(kNumBatchShapes - 1, std::atoi(e)));
  } else {
    bool have_status = true;
    for (auto &p : pr) have_status &= p.status_out != nullptr;
    if (have_status) {
      shape = tune(ctx, pr, bf16);
      if (shape < 0) return VG_EDEVICE;
    }
  }
  // key: everything the launches depend on
  int64_t items0, rays0;
  std::vector<BatchProblem> probe =
      make_table(pr, order, shape, bf16, nullptr, nullptr, nullptr, items0, rays0);
  uint64_t key = fnv(probe.data(), probe.size() * sizeof(BatchProblem));
  key = fnv(&shape, sizeof shape, key);
  key = fnv(&flags, sizeof flags, key);
  bool need_status = false;
  for (auto &p : pr) need_status |= p.status_out == nullptr;
  // item range of each register class (the table is grouped by class)
  int64_t cls_first[kNumBatchClasses], cls_last[kNumBatchClasses];
  for (int c = 0; c < kNumBatchClasses; ++c) cls_first[c] = cls_last[c] = 0;
  for (size_t q = 0; q < probe.size(); ++q) {
    const int c = batched_class(probe[q].a.d, bf16);
    const int64_t b0 = probe[q].item_begin;
    const int64_t b1 = q + 1 < probe.size() ? probe[q + 1].item_begin : items0;
    if (cls_last[c] == cls_first[c]) cls_first[c] = b0;
    cls_last[c] = b1;
  }
  auto fill = [&](const BatchBuffers &b, std::vector<char> &bytes) {
    int64_t items, rays;
    std::vector<BatchProblem> T =
        make_table(pr, order, shape, bf16, b.counters, b.flags, b.status, items, rays);
    bytes.assign(reinterpret_cast<const char *>(T.data()),
                 reinterpret_cast<const char *>(T.data() + T.size()));
  };
  auto enqueue = [&](const BatchBuffers &b, hipStream_t s) -> hipError_t {
    const int rgrid = (int)std::min<int64_t>((rays0 + 3) / 4, 2048);
    unsigned long long *next = reinterpret_cast<unsigned long long *>((char *)b.counters + 32);
    hipError_t e = fill_u32(b.counters, 0u, 16, s);
    for (int c = 0; c < kNumBatchClasses && e == hipSuccess; ++c) {
      if (cls_last[c] <= cls_first[c]) continue;
      const int grid = (int)std::min<int64_t>(cls_last[c] - cls_first[c], persistent_grid(ctx, shape, bf16, c));
      e = launch_cell_scan_batched((const BatchProblem *)b.table, n_problems, cls_first[c], cls_last[c],
                                   next + c, shape, bf16, c, grid, s);
    }
    if (e == hipSuccess)
      e = launch_recheck_batched((const BatchProblem *)b.table, b.counters, b.flags,
                                 b.counters + CNT_FP64_TIE, std::max(rgrid, 1), s);
    return e;
  };
  return run_batch(ctx, key, rays0, need_status, probe.size() * sizeof(BatchProblem), fill, enqueue,
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
    unsigned long long *next = reinterpret_cast<unsigned long long *>((char *)b.counters + 32);
    hipError_t e = fill_u32(b.counters, 0u, 16, s);
    if (e == hipSuccess)
      e = launch_ray_scan_batched((const RayBatchProblem *)b.table, np, items0, next, grid, s);
    if (e == hipSuccess)
      e = launch_recheck_rays_batched((const RayBatchProblem *)b.table, b.counters, b.flags,
                                      b.counters + CNT_FP64_TIE, std::max(rgrid, 1), s);
    return e;
  };
  return run_batch(ctx, key, rays0, need_status, probe.size() * sizeof(RayBatchProblem), fill,
                   enqueue, kTauRays);
}
