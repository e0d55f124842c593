// C ABI entry points: argument validation, scratch management and kernel
// sequencing.  No arithmetic of the method happens here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "vg_explore.h"
#include "vg_internal.h"

using namespace vg;

namespace {

int fail(vg_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(vg_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_fail(vg_ctx *ctx, hipError_t e, const char *what) {
  return fail(ctx, VG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define VG_HIP(ctx, call)                          \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Carve a 256-byte aligned block out of the context scratch.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
  static size_t need(std::initializer_list<size_t> bytes) {
    size_t s = 0;
    for (size_t b : bytes) s = ((s + 255) & ~size_t(255)) + b;
    return s + 256;
  }
};

// Grow the context scratch.  The old block is not freed but kept until
// vg_destroy: a call captured into a graph earlier still reads it.  Growing
// at least twofold bounds the kept blocks by the live one.
int ensure_scratch(vg_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return VG_OK;
  const size_t want = std::max(bytes + bytes / 4, 2 * ctx->scratch_bytes);
  void *p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, VG_ENOMEM, "scratch allocation of %zu bytes failed", want);
  }
  if (ctx->scratch) ctx->retired.push_back(ctx->scratch);
  ctx->scratch = p;
  ctx->scratch_bytes = want;
  return VG_OK;
}

int check_common(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes) {
  if (!ctx) return VG_EINVAL;
  ctx->err.clear();
  if (d < 2 || d > VG_MAX_DIM) return fail(ctx, VG_EUNSUPPORTED, "d=%d outside [2, %d]", d, VG_MAX_DIM);
  if (n_nodes < 1 || n_nodes >= (int64_t(1) << 31))
    return fail(ctx, VG_EINVAL, "n_nodes=%lld outside [1, 2^31)", (long long)n_nodes);
  if (!nodes) return fail(ctx, VG_EINVAL, "nodes is NULL");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VG_EDEVICE, "hipSetDevice failed");
  return VG_OK;
}

// Event pair around a scan launch when profiling (recorded on ctx->stream).
struct ScanTimer {
  vg_ctx *ctx;
  hipEvent_t a = nullptr, b = nullptr;
  explicit ScanTimer(vg_ctx *c, bool enable = true) : ctx(c) {
    if (!enable || !ctx->profiling) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      ctx->profiling = false;
      return;
    }
    (void)hipEventRecord(a, ctx->stream);
  }
  void stop() {
    if (!a) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->scan_events.emplace_back(a, b);
    a = b = nullptr;
  }
};

double sphere_area(int d) { return 2.0 * std::pow(M_PI, 0.5 * d) / std::tgamma(0.5 * d); }

}  // namespace

namespace vg {

int run_cells_in(vg_ctx *ctx, int d, int64_t n, const float *nodes, int R, const float *dirs,
                 uint64_t seed, uint32_t flags, float *t_out, int32_t *idx_out, const CellsScratch &sc,
                 const int64_t *nbr_off, const int32_t *nbr) {
  const int64_t m = n * (int64_t)R;
  const bool recheck = !(flags & VG_NO_RECHECK);
  const bool bf16 = (flags & VG_PREC_BF16X3) != 0;
  const bool incircle = (flags & VG_INCIRCLE) != 0;
  int64_t *flag_list = recheck ? sc.flag_list : nullptr;
  uint8_t *st = sc.status;
  void *grid_scratch = sc.grid;
  void *parts = sc.parts;
  const size_t parts_bytes = sc.parts_bytes;
  ctx->last_counters = sc.counters;
  VG_HIP(ctx, fill_u32(sc.counters, 0u, CNT_WORDS, ctx->stream));
  VG_HIP(ctx, launch_check_finite(nodes, n * d, sc.counters + CNT_BAD_NODES, ctx->stream));

  CellScanArgs a{};
  a.nodes = nodes;
  a.n = n;
  a.d = d;
  a.dirs = dirs;
  a.seed = seed;
  a.R = R;
  if (sc.xs && !nbr && !incircle) {
    VG_HIP(ctx, launch_node_order(nodes, n, d, sc.order_keys, sc.perm, sc.rank, sc.xs, sc.aabb, ctx->stream));
    a.xs = sc.xs;
    a.perm = sc.perm;
    a.rank = sc.rank;
    a.aabb = sc.aabb;
  }
  a.t_out = t_out;
  a.idx_out = idx_out;
  a.st_out = st;
  a.counters = sc.counters;
  a.flag_list = flag_list;
  a.tau_rel = bf16 ? kTauCellsBf16 : kTauCellsFp32;
  a.kappa = cell_kappa(d, bf16);
  a.nbr_off = nbr_off;
  a.nbr = nbr;
  ScanTimer timer(ctx, sc.timed);
  hipError_t e;
  if (incircle)
    e = launch_incircle_cells(a, grid_scratch,
                              reinterpret_cast<unsigned long long *>(sc.counters + CNT_NN_CALLS), ctx->stream);
  else
    e = bf16 ? launch_cell_scan_bf16x3(a, ctx->stream) : launch_cell_scan_fp32(a, ctx->stream);
  timer.stop();
  if (e != hipSuccess) return hip_fail(ctx, e, "cell scan launch");
  if (recheck) {
    RecheckArgs r{};
    r.mode = RAYS_CELLS;
    r.nodes = nodes;
    r.n = n;
    r.d = d;
    r.dirs = dirs;
    r.seed = seed;
    r.R = R;
    r.clip = 1;
    r.counters = sc.counters;
    r.flag_list = flag_list;
    r.t_out = t_out;
    r.idx_out = idx_out;
    r.st_out = st;
    r.tie_counter = sc.counters + CNT_FP64_TIE;
    if (!launch_recheck_cells_split(r, m, parts, parts_bytes, ctx->stream, e))
      e = launch_recheck(r, (int)std::min<int64_t>(m, 4096), ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "recheck launch");
  }
  if (incircle) {
    // the dense scans answer rays with non-finite input themselves; the
    // incircle kernels stop at a non-finite node and leave it to this pass
    FinalizeArgs f{};
    f.m = m;
    f.d = d;
    f.u32 = dirs;
    f.flags = sc.counters;
    f.bad_rays = sc.counters + CNT_BAD_RAYS;
    f.t_out = t_out;
    f.idx_out = idx_out;
    f.st_out = st;
    VG_HIP(ctx, launch_finalize_bad(f, ctx->stream));
  }
  ctx->last_rays = m;
  ctx->last_tau = a.tau_rel;
  return VG_OK;
}

}  // namespace vg

namespace {

// run_cells_in with the scratch carved out of the context's (grown on demand).
int run_cells(vg_ctx *ctx, int d, int64_t n, const float *nodes, int R, const float *dirs, uint64_t seed,
              uint32_t flags, float *t_out, int32_t *idx_out, uint8_t *st_out,
              const int64_t *nbr_off = nullptr, const int32_t *nbr = nullptr) {
  const int64_t m = n * (int64_t)R;
  const bool recheck = !(flags & VG_NO_RECHECK);
  const bool bf16 = (flags & VG_PREC_BF16X3) != 0;
  const bool incircle = (flags & VG_INCIRCLE) != 0;
  if (incircle && (bf16 || nbr || d > 6 || !dirs))
    return fail(ctx, VG_EUNSUPPORTED,
                "VG_INCIRCLE needs d <= 6, FP32, no neighbour lists and directions as input");
  const size_t grid_bytes = incircle ? incircle_scratch_bytes(n, d, R) : 0;
  const size_t parts_bytes = recheck ? recheck_cells_reserve(m, n) : 0;
  if ((flags & VG_SCAN_ORDER) && (flags & VG_INDEX_ORDER))
    return fail(ctx, VG_EINVAL, "VG_SCAN_ORDER and VG_INDEX_ORDER exclude each other");
  const bool ordered = !incircle && !nbr && scan_order(d, flags, bf16);
  const int64_t n_keys = ordered ? node_order_keys(n) : 0;
  size_t need = Carver::need({recheck ? (size_t)m * 8 : 0, st_out ? 0 : (size_t)m, grid_bytes, parts_bytes,
                              (size_t)n_keys * 8, ordered ? (size_t)n * 4 : 0, ordered ? (size_t)n * 4 : 0,
                              ordered ? (size_t)(n * d) * 4 : 0,
                              ordered ? (size_t)order_box_floats(n, d) * 4 : 0});
  int rc = ensure_scratch(ctx, need);
  if (rc) return rc;
  Carver cv(ctx->scratch);
  CellsScratch sc{};
  if (ordered) {
    sc.order_keys = cv.take<uint64_t>(n_keys);
    sc.perm = cv.take<int32_t>(n);
    sc.rank = cv.take<int32_t>(n);
    sc.xs = cv.take<float>(n * d);
    sc.aabb = cv.take<float>(order_box_floats(n, d));
  }
  sc.flag_list = recheck ? cv.take<int64_t>(m) : nullptr;
  sc.status = st_out ? st_out : cv.take<uint8_t>(m);
  sc.grid = incircle ? cv.take<char>(grid_bytes) : nullptr;
  sc.parts = parts_bytes ? cv.take<char>(parts_bytes) : nullptr;
  sc.parts_bytes = parts_bytes;
  sc.counters = ctx->counters;
  sc.timed = true;
  return run_cells_in(ctx, d, n, nodes, R, dirs, seed, flags, t_out, idx_out, sc, nbr_off, nbr);
}

}  // namespace

namespace vg {

int raycast_f64(vg_ctx *ctx, int d, int64_t n, const float *nodes, int64_t m, const double *o64,
                const double *u64, const int32_t *gen, const int32_t *excl, int n_excl, int clip,
                bool force_all, float *t_out, int32_t *idx_out, uint8_t *st_out, double *t64,
                int incircle, const double *nodes64, float node_err, bool check_input) {
  if (m <= 0) return VG_OK;
  if (nodes64 && incircle) return fail(ctx, VG_EUNSUPPORTED, "exact FP64 rows need the dense scan");
  const size_t grid_bytes = incircle ? incircle_rays_scratch_bytes(n, d) : 0;
  const size_t split_bytes = incircle ? 0 : ray_scan_split_bytes(m, n);
  const size_t parts_bytes = recheck_split_reserve(m, n);
  size_t need = Carver::need({(size_t)m * 8, grid_bytes, split_bytes, parts_bytes, st_out ? 0 : (size_t)m});
  int rc = ensure_scratch(ctx, need);
  if (rc) return rc;
  Carver cv(ctx->scratch);
  int64_t *flag_list = cv.take<int64_t>(m);
  void *grid_scratch = incircle ? cv.take<char>(grid_bytes) : nullptr;
  void *split = split_bytes ? cv.take<char>(split_bytes) : nullptr;
  void *parts = parts_bytes ? cv.take<char>(parts_bytes) : nullptr;
  if (!st_out) st_out = cv.take<uint8_t>(m);
  ctx->last_counters = ctx->counters;
  VG_HIP(ctx, fill_u32(ctx->counters, 0u, CNT_WORDS, ctx->stream));
  if (check_input) VG_HIP(ctx, launch_check_finite(nodes, n * d, ctx->counters + CNT_BAD_NODES, ctx->stream));
  RayScanArgs a{};
  a.nodes = nodes;
  a.n = n;
  a.d = d;
  a.m = m;
  a.o64 = o64;
  a.u64 = u64;
  a.gen = gen;
  a.excl = excl;
  a.n_excl = n_excl;
  a.clip = clip;
  a.t_out = t_out;
  a.idx_out = idx_out;
  a.st_out = st_out;
  a.counters = ctx->counters;
  a.flag_list = flag_list;
  a.tau = kTauRays;
  a.force_all = force_all ? 1 : 0;
  a.node_err = nodes64 ? node_err : 0.f;
  ScanTimer timer(ctx);
  hipError_t e =
      incircle ? launch_incircle_rays(a, grid_scratch, incircle == 2,
                                      reinterpret_cast<unsigned long long *>(ctx->counters + CNT_NN_CALLS),
                                      ctx->stream)
               : launch_ray_scan(a, split, split_bytes, ctx->stream);
  timer.stop();
  if (e != hipSuccess) return hip_fail(ctx, e, "ray scan launch");
  RecheckArgs r{};
  r.mode = RAYS_F64;
  r.nodes = nodes;
  r.n = n;
  r.d = d;
  r.o64 = o64;
  r.u64 = u64;
  r.gen = gen;
  r.excl = excl;
  r.n_excl = n_excl;
  r.clip = clip;
  r.counters = ctx->counters;
  r.flag_list = flag_list;
  r.t_out = t_out;
  r.idx_out = idx_out;
  r.st_out = st_out;
  r.tie_counter = ctx->counters + CNT_FP64_TIE;
  r.t64_out = t64;
  r.nodes64 = nodes64;
  // the queue length, read here (callers of this path synchronise anyway),
  // sizes a split recheck over many nodes
  uint32_t queued = 0;
  VG_HIP(ctx, hipMemcpyAsync(&queued, ctx->counters + CNT_FLAGGED, 4, hipMemcpyDeviceToHost, ctx->stream));
  VG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (queued > 0 && !launch_recheck_split(r, queued, parts, parts_bytes, ctx->stream, e))
    e = launch_recheck(r, (int)std::min<int64_t>(m, 4096), ctx->stream, queued);
  if (e != hipSuccess) return hip_fail(ctx, e, "recheck launch");
  if (check_input) {
    FinalizeArgs f{};
    f.m = m;
    f.d = d;
    f.o64 = o64;
    f.u64 = u64;
    f.flags = ctx->counters;
    f.bad_rays = ctx->counters + CNT_BAD_RAYS;
    f.t_out = t_out;
    f.idx_out = idx_out;
    f.st_out = st_out;
    VG_HIP(ctx, launch_finalize_bad(f, ctx->stream));
  }
  ctx->last_rays = m;
  ctx->last_tau = kTauRays;
  return VG_OK;
}

}  // namespace vg

extern "C" {

int vg_create(int device, vg_ctx **out) {
  if (!out) return VG_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return VG_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return VG_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return VG_EDEVICE;
  vg_ctx *ctx = new (std::nothrow) vg_ctx();
  if (!ctx) return VG_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipMalloc(&ctx->counters, CNT_WORDS * sizeof(uint32_t)) != hipSuccess) {
    delete ctx;
    return VG_EDEVICE;
  }
  // the fixed scratch of vg_raycast_cells_noalloc on this device (looked up
  // once per device, with the device current)
  if (noalloc_attach(device) != hipSuccess) {
    (void)hipFree(ctx->counters);
    delete ctx;
    return VG_EDEVICE;
  }
  *out = ctx;
  return VG_OK;
}

void vg_destroy(vg_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &ev : ctx->scan_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  batch_state_free(ctx);
  if (ctx->handoff) (void)hipEventDestroy(ctx->handoff);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  for (void *p : ctx->retired) (void)hipFree(p);
  if (ctx->counters) (void)hipFree(ctx->counters);
  delete ctx;
}

int vg_set_stream(vg_ctx *ctx, void *stream) {
  if (!ctx) return VG_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (s == ctx->stream) return VG_OK;
  // Every call of a context shares its counters, its scratch (recheck queue,
  // split partials) and the batch buffers, so work enqueued on the new stream
  // must not start before the old stream has finished this context's earlier
  // calls: the new stream waits for an event recorded on the old one.
  VG_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->handoff) VG_HIP(ctx, hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming));
  if (hipEventRecord(ctx->handoff, ctx->stream) == hipSuccess) {
    VG_HIP(ctx, hipStreamWaitEvent(s, ctx->handoff, 0));
  } else {
    // the old stream cannot take an event (e.g. it was destroyed): wait for
    // all work on the device instead
    (void)hipGetLastError();
    VG_HIP(ctx, hipDeviceSynchronize());
  }
  ctx->stream = s;
  return VG_OK;
}

const char *vg_last_error(const vg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int vg_get_stats(vg_ctx *ctx, vg_stats *out) {
  if (!ctx || !out) return VG_EINVAL;
  uint32_t c[CNT_WORDS];
  VG_HIP(ctx, hipSetDevice(ctx->device));
  VG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  VG_HIP(ctx, hipMemcpy(c, ctx->last_counters ? ctx->last_counters : ctx->counters, sizeof c,
                        hipMemcpyDeviceToHost));
  out->rays = ctx->last_rays;
  out->nn_calls = (int64_t)((uint64_t)c[CNT_NN_CALLS] | ((uint64_t)c[CNT_NN_CALLS + 1] << 32));
  out->nn_grid_calls = (int64_t)((uint64_t)c[CNT_NN_GRID] | ((uint64_t)c[CNT_NN_GRID + 1] << 32));
  out->flagged = c[CNT_FLAGGED];
  out->fp64_ties = c[CNT_FP64_TIE];
  out->bad_input_rays = c[CNT_BAD_RAYS];
  out->bad_node_values = c[CNT_BAD_NODES];
  out->scan_pairs = (int64_t)(((uint64_t)c[CNT_SCAN_BLOCKS] | ((uint64_t)c[CNT_SCAN_BLOCKS + 1] << 32)) * 1024u);
  out->tie_eps = ctx->last_tau;
  for (auto &ev : ctx->scan_events) {
    float ms = 0.f;
    VG_HIP(ctx, hipEventElapsedTime(&ms, ev.first, ev.second));
    ctx->scan_ms += ms;
    ctx->scan_launches++;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  ctx->scan_events.clear();
  out->scan_launches = ctx->scan_launches;
  out->scan_ms = ctx->scan_ms;
  return VG_OK;
}

int vg_set_profiling(vg_ctx *ctx, int enable) {
  if (!ctx) return VG_EINVAL;
  VG_HIP(ctx, hipSetDevice(ctx->device));
  VG_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto &ev : ctx->scan_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  ctx->scan_events.clear();
  ctx->scan_launches = 0;
  ctx->scan_ms = 0.0;
  ctx->profiling = enable != 0;
  return VG_OK;
}

int vg_raycast(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_rays,
               const float *origin, const float *dir, const int32_t *gen, const int32_t *excl,
               int n_excl, uint32_t flags, float *t_out, int32_t *idx_out, uint8_t *status_out) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (n_rays < 0) return fail(ctx, VG_EINVAL, "n_rays < 0");
  if (n_excl < 0 || n_excl > d) return fail(ctx, VG_EINVAL, "n_excl=%d outside [0, d]", n_excl);
  if (n_rays == 0) return VG_OK;
  if (!origin || !dir || !gen || !t_out || !idx_out) return fail(ctx, VG_EINVAL, "null ray array");
  if (n_excl > 0 && !excl) return fail(ctx, VG_EINVAL, "excl is NULL with n_excl > 0");
  const bool recheck = !(flags & VG_NO_RECHECK);
  const bool incircle = (flags & VG_INCIRCLE) != 0;
  if (incircle && d > 6) return fail(ctx, VG_EUNSUPPORTED, "VG_INCIRCLE needs d <= 6");
  if ((flags & VG_INIT_HEURISTIC) && !incircle)
    return fail(ctx, VG_EINVAL, "VG_INIT_HEURISTIC needs VG_INCIRCLE");
  const size_t grid_bytes = incircle ? incircle_rays_scratch_bytes(n_nodes, d) : 0;
  const size_t split_bytes = incircle ? 0 : ray_scan_split_bytes(n_rays, n_nodes);
  size_t need = Carver::need(
      {recheck ? (size_t)n_rays * 8 : 0, status_out ? 0 : (size_t)n_rays, grid_bytes, split_bytes});
  rc = ensure_scratch(ctx, need);
  if (rc) return rc;
  Carver cv(ctx->scratch);
  int64_t *flag_list = recheck ? cv.take<int64_t>(n_rays) : nullptr;
  uint8_t *st = status_out ? status_out : cv.take<uint8_t>(n_rays);
  void *grid_scratch = incircle ? cv.take<char>(grid_bytes) : nullptr;
  void *split = split_bytes ? cv.take<char>(split_bytes) : nullptr;
  ctx->last_counters = ctx->counters;
  VG_HIP(ctx, fill_u32(ctx->counters, 0u, CNT_WORDS, ctx->stream));
  VG_HIP(ctx, launch_check_finite(nodes, n_nodes * d, ctx->counters + CNT_BAD_NODES, ctx->stream));
  RayScanArgs a{};
  a.nodes = nodes;
  a.n = n_nodes;
  a.d = d;
  a.m = n_rays;
  a.o32 = origin;
  a.u32 = dir;
  a.gen = gen;
  a.excl = excl;
  a.n_excl = n_excl;
  a.clip = (flags & VG_CLIP) ? 1 : 0;
  a.t_out = t_out;
  a.idx_out = idx_out;
  a.st_out = st;
  a.counters = ctx->counters;
  a.flag_list = flag_list;
  a.tau = kTauRays;
  ScanTimer timer(ctx);
  hipError_t e =
      incircle ? launch_incircle_rays(a, grid_scratch, (flags & VG_INIT_HEURISTIC) ? 1 : 0,
                                      reinterpret_cast<unsigned long long *>(ctx->counters + CNT_NN_CALLS),
                                      ctx->stream)
               : launch_ray_scan(a, split, split_bytes, ctx->stream);
  timer.stop();
  if (e != hipSuccess) return hip_fail(ctx, e, "ray scan launch");
  if (recheck) {
    RecheckArgs r{};
    r.mode = RAYS_F32;
    r.nodes = nodes;
    r.n = n_nodes;
    r.d = d;
    r.o32 = origin;
    r.u32 = dir;
    r.gen = gen;
    r.excl = excl;
    r.n_excl = n_excl;
    r.clip = a.clip;
    r.counters = ctx->counters;
    r.flag_list = flag_list;
    r.t_out = t_out;
    r.idx_out = idx_out;
    r.st_out = st;
    r.tie_counter = ctx->counters + CNT_FP64_TIE;
    e = launch_recheck(r, (int)std::min<int64_t>(n_rays, 4096), ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "recheck launch");
  }
  FinalizeArgs f{};
  f.m = n_rays;
  f.d = d;
  f.o32 = origin;
  f.u32 = dir;
  f.flags = ctx->counters;
  f.bad_rays = ctx->counters + CNT_BAD_RAYS;
  f.t_out = t_out;
  f.idx_out = idx_out;
  f.st_out = st;
  VG_HIP(ctx, launch_finalize_bad(f, ctx->stream));
  ctx->last_rays = n_rays;
  ctx->last_tau = kTauRays;
  return VG_OK;
}

int vg_raycast_f64(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_rays,
                   const double *origin, const double *dir, const int32_t *gen, const int32_t *excl, int n_excl,
                   uint32_t flags, float *t_out, int32_t *idx_out, uint8_t *status_out) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (n_rays < 0) return fail(ctx, VG_EINVAL, "n_rays < 0");
  if (n_excl < 0 || n_excl > d) return fail(ctx, VG_EINVAL, "n_excl=%d outside [0, d]", n_excl);
  if (n_rays == 0) return VG_OK;
  if (!origin || !dir || !gen || !t_out || !idx_out) return fail(ctx, VG_EINVAL, "null ray array");
  if (n_excl > 0 && !excl) return fail(ctx, VG_EINVAL, "excl is NULL with n_excl > 0");
  if (flags & ~(uint32_t)(VG_CLIP | VG_INCIRCLE | VG_INIT_HEURISTIC))
    return fail(ctx, VG_EINVAL, "vg_raycast_f64 takes VG_CLIP, VG_INCIRCLE and VG_INIT_HEURISTIC only");
  const bool incircle = (flags & VG_INCIRCLE) != 0;
  if (incircle && d > 6) return fail(ctx, VG_EUNSUPPORTED, "VG_INCIRCLE needs d <= 6");
  if ((flags & VG_INIT_HEURISTIC) && !incircle)
    return fail(ctx, VG_EINVAL, "VG_INIT_HEURISTIC needs VG_INCIRCLE");
  return raycast_f64(ctx, d, n_nodes, nodes, n_rays, origin, dir, gen, excl, n_excl, (flags & VG_CLIP) ? 1 : 0,
                     false, t_out, idx_out, status_out, nullptr,
                     incircle ? ((flags & VG_INIT_HEURISTIC) ? 2 : 1) : 0, nullptr, 0.f, true);
}

int vg_raycast_cells(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                     const float *dirs, uint32_t flags, float *t_out, int32_t *idx_out,
                     uint8_t *status_out) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (!dirs || !t_out || !idx_out) return fail(ctx, VG_EINVAL, "null array");
  return run_cells(ctx, d, n_nodes, nodes, rays_per_cell, dirs, 0, flags, t_out, idx_out, status_out);
}

int vg_raycast_cells_noalloc(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                             const float *dirs, uint32_t flags, float *t_out, int32_t *idx_out,
                             uint8_t *status_out) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (!dirs || !t_out || !idx_out) return fail(ctx, VG_EINVAL, "null array");
  if (flags & VG_INCIRCLE) return fail(ctx, VG_EUNSUPPORTED, "VG_INCIRCLE needs scratch of its own");
  if (flags & VG_SCAN_ORDER) return fail(ctx, VG_EUNSUPPORTED, "VG_SCAN_ORDER needs scratch of its own");
  const int64_t m = n_nodes * (int64_t)rays_per_cell;
  if (m > VG_NOALLOC_MAX_RAYS)
    return fail(ctx, VG_EINVAL, "n_nodes * rays_per_cell = %lld exceeds VG_NOALLOC_MAX_RAYS = %lld",
                (long long)m, (long long)VG_NOALLOC_MAX_RAYS);
  static_assert(VG_NOALLOC_MAX_RAYS == kNoAllocMaxRays, "header and library disagree");
  char *base = static_cast<char *>(noalloc_scratch(ctx->device));
  if (!base) return fail(ctx, VG_EDEVICE, "fixed scratch not attached on device %d", ctx->device);
  // layout: counters | recheck queue [m] i64 | status [m] u8
  CellsScratch sc{};
  sc.counters = reinterpret_cast<uint32_t *>(base);
  sc.flag_list = reinterpret_cast<int64_t *>(base + kNoAllocCounterBytes);
  sc.status = status_out ? status_out
                         : reinterpret_cast<uint8_t *>(base + kNoAllocCounterBytes + (size_t)kNoAllocMaxRays * 8);
  sc.timed = false;
  return run_cells_in(ctx, d, n_nodes, nodes, rays_per_cell, dirs, 0, flags, t_out, idx_out, sc, nullptr,
                      nullptr);
}

}  // extern "C"

namespace {

int mc_volume_area(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, const int64_t *nbr_off,
                   const int32_t *nbr, int rays_per_cell, const float *dirs, uint64_t seed, bool seeded,
                   uint32_t flags,
                   float *t_out, int32_t *idx_out, uint8_t *status_out, float *volume,
                   float *energy2, int32_t *facet_j, float *facet_area, int32_t *facet_count) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if ((!dirs && !seeded) || !t_out || !idx_out || !volume) return fail(ctx, VG_EINVAL, "null array");
  const int nf = (facet_j != nullptr) + (facet_area != nullptr) + (facet_count != nullptr);
  if (nf != 0 && nf != 3) return fail(ctx, VG_EINVAL, "facet outputs must be all set or all NULL");
  rc = run_cells(ctx, d, n_nodes, nodes, rays_per_cell, seeded ? nullptr : dirs, seed, flags, t_out, idx_out,
                 status_out, nbr_off, nbr);
  if (rc) return rc;
  const double S = sphere_area(d);
  AccumArgs a{};
  a.nodes = nodes;
  a.n = n_nodes;
  a.d = d;
  a.R = rays_per_cell;
  a.t = t_out;
  a.idx = idx_out;
  a.sv = (float)(S / ((double)d * rays_per_cell));
  a.se = (float)(S / ((double)(d + 2) * rays_per_cell));
  a.sa = (float)(S / (double)rays_per_cell);
  a.volume = volume;
  a.energy2 = energy2;
  a.facet_j = facet_j;
  a.facet_area = facet_area;
  a.facet_count = facet_count;
  hipError_t e = launch_accum(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "accumulate launch");
  return VG_OK;
}

}  // namespace

extern "C" {

int vg_mc_volume_area(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                      const float *dirs, uint32_t flags, float *t_out, int32_t *idx_out,
                      uint8_t *status_out, float *volume, float *energy2, int32_t *facet_j,
                      float *facet_area, int32_t *facet_count) {
  return mc_volume_area(ctx, d, n_nodes, nodes, nullptr, nullptr, rays_per_cell, dirs, 0, false, flags, t_out,
                        idx_out, status_out, volume, energy2, facet_j, facet_area, facet_count);
}

int vg_mc_volume_area_nbr(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes,
                          const int64_t *nbr_offsets, const int32_t *nbr, int rays_per_cell,
                          const float *dirs, uint32_t flags, float *t_out, int32_t *idx_out,
                          uint8_t *status_out, float *volume, float *energy2, int32_t *facet_j,
                          float *facet_area, int32_t *facet_count) {
  if (!ctx) return VG_EINVAL;
  if (!nbr_offsets || !nbr) return fail(ctx, VG_EINVAL, "nbr_offsets and nbr are required");
  return mc_volume_area(ctx, d, n_nodes, nodes, nbr_offsets, nbr, rays_per_cell, dirs, 0, false, flags, t_out,
                        idx_out, status_out, volume, energy2, facet_j, facet_area, facet_count);
}

int vg_raycast_cells_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                            uint64_t seed, uint32_t flags, float *t_out, int32_t *idx_out, uint8_t *status_out) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (!t_out || !idx_out) return fail(ctx, VG_EINVAL, "null array");
  return run_cells(ctx, d, n_nodes, nodes, rays_per_cell, nullptr, seed, flags, t_out, idx_out, status_out);
}

int vg_mc_volume_area_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                             uint64_t seed, uint32_t flags, float *t_out, int32_t *idx_out,
                             uint8_t *status_out, float *volume, float *energy2, int32_t *facet_j,
                             float *facet_area, int32_t *facet_count) {
  return mc_volume_area(ctx, d, n_nodes, nodes, nullptr, nullptr, rays_per_cell, nullptr, seed, true, flags,
                        t_out, idx_out, status_out, volume, energy2, facet_j, facet_area, facet_count);
}

int vg_dump_dirs(vg_ctx *ctx, int d, int64_t first_cell, int64_t n_cells, int rays_per_cell, uint64_t seed,
                 float *out) {
  if (!ctx) return VG_EINVAL;
  ctx->err.clear();
  if (d < 2 || d > VG_MAX_DIM) return fail(ctx, VG_EUNSUPPORTED, "d=%d outside [2, %d]", d, VG_MAX_DIM);
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (first_cell < 0 || n_cells < 0 || first_cell + n_cells > (int64_t(1) << 31))
    return fail(ctx, VG_EINVAL, "cells [%lld, %lld) outside [0, 2^31)", (long long)first_cell,
                (long long)(first_cell + n_cells));
  if (n_cells == 0) return VG_OK;
  if (!out) return fail(ctx, VG_EINVAL, "out is NULL");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VG_EDEVICE, "hipSetDevice failed");
  VG_HIP(ctx, launch_dump_dirs(d, first_cell, n_cells, rays_per_cell, seed, out, ctx->stream));
  return VG_OK;
}

int vg_mc_sample_points(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                        const float *dirs, const float *t, int m, const float *tsamp, float *points) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (m < 0 || m > 1024) return fail(ctx, VG_EINVAL, "m=%d outside [0, 1024]", m);
  if (!dirs || !t || !points || (m > 0 && !tsamp)) return fail(ctx, VG_EINVAL, "null array");
  VG_HIP(ctx, launch_sample_points(nodes, n_nodes, d, rays_per_cell, dirs, t, m, tsamp, points, ctx->stream));
  return VG_OK;
}

int vg_mc_integrals(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                    const float *t, const int32_t *idx, int m, const float *tsamp, const float *fvals,
                    float *fint_volume, int32_t *facet_j, float *fint_facet, int32_t *facet_count) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (m < 0 || m > 1024) return fail(ctx, VG_EINVAL, "m=%d outside [0, 1024]", m);
  if (!t || !idx || !fvals || (m > 0 && !tsamp)) return fail(ctx, VG_EINVAL, "null array");
  const int nf = (facet_j != nullptr) + (fint_facet != nullptr) + (facet_count != nullptr);
  if (nf != 0 && nf != 3) return fail(ctx, VG_EINVAL, "facet outputs must be all set or all NULL");
  if (m > 0 && !fint_volume) return fail(ctx, VG_EINVAL, "fint_volume is NULL with m > 0");
  const double S = sphere_area(d);
  AccumArgs a{};
  a.nodes = nodes;
  a.n = n_nodes;
  a.d = d;
  a.R = rays_per_cell;
  a.t = t;
  a.idx = idx;
  a.sa = (float)(S / (double)rays_per_cell);
  a.facet_j = facet_j;
  a.facet_count = facet_count;
  a.m = m;
  a.tsamp = tsamp;
  a.fvals = fvals;
  a.sf = m > 0 ? (float)(S / ((double)rays_per_cell * m)) : 0.f;
  a.fint_volume = m > 0 ? fint_volume : nullptr;
  a.fint_facet = fint_facet;
  VG_HIP(ctx, launch_accum(a, ctx->stream));
  return VG_OK;
}

static int hmc_check(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_vertices,
                     const int32_t *sigma, int rays_per_cell, const int32_t *facet_j,
                     const int32_t *facet_count) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if (n_vertices < 0 || (n_vertices > 0 && !sigma)) return fail(ctx, VG_EINVAL, "bad vertex array");
  if (n_nodes + 2 * d >= (int64_t(1) << 31)) return fail(ctx, VG_EINVAL, "n_nodes too large for int32 keys");
  if (!facet_j || !facet_count) return fail(ctx, VG_EINVAL, "null facet array");
  return VG_OK;
}

int vg_hmc_centroids(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_vertices,
                     const int32_t *sigma, const double *coords, int rays_per_cell, const int32_t *facet_j,
                     const int32_t *facet_count, float *centroid, int32_t *kcount) {
  int rc = hmc_check(ctx, d, n_nodes, nodes, n_vertices, sigma, rays_per_cell, facet_j, facet_count);
  if (rc) return rc;
  if (!coords || !centroid || !kcount) return fail(ctx, VG_EINVAL, "null array");
  return hmc_run(false, d, n_nodes, nodes, n_vertices, sigma, coords, nullptr, rays_per_cell, facet_j, nullptr,
                 facet_count, nullptr, nullptr, centroid, kcount, nullptr, nullptr, nullptr, ctx->stream,
                 ctx->err);
}

int vg_hmc_integrals(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int64_t n_vertices,
                     const int32_t *sigma, const float *f_vertex, int rays_per_cell, const int32_t *facet_j,
                     const float *facet_area, const int32_t *facet_count, const float *f_centroid,
                     const float *f_node, float *fint_facet, float *fint_cell, float *volume) {
  int rc = hmc_check(ctx, d, n_nodes, nodes, n_vertices, sigma, rays_per_cell, facet_j, facet_count);
  if (rc) return rc;
  if (!f_vertex || !facet_area || !f_centroid || !f_node || !fint_facet || !fint_cell || !volume)
    return fail(ctx, VG_EINVAL, "null array");
  return hmc_run(true, d, n_nodes, nodes, n_vertices, sigma, nullptr, f_vertex, rays_per_cell, facet_j,
                 facet_area, facet_count, f_centroid, f_node, nullptr, nullptr, fint_facet, fint_cell, volume,
                 ctx->stream, ctx->err);
}

int vg_tuple_neighbors(vg_ctx *ctx, int d, int64_t n_nodes, int64_t n_tuples, const int32_t *sigma,
                       int64_t *offsets, int32_t *nbr, int64_t nbr_capacity, int64_t *nnz) {
  if (!ctx) return VG_EINVAL;
  ctx->err.clear();
  if (d < 2 || d > VG_MAX_DIM) return fail(ctx, VG_EUNSUPPORTED, "d=%d outside [2, %d]", d, VG_MAX_DIM);
  if (n_nodes < 1 || n_nodes >= (int64_t(1) << 31))
    return fail(ctx, VG_EINVAL, "n_nodes=%lld outside [1, 2^31)", (long long)n_nodes);
  if (n_tuples < 0 || (n_tuples > 0 && !sigma)) return fail(ctx, VG_EINVAL, "bad tuple array");
  if (!nnz) return fail(ctx, VG_EINVAL, "nnz is NULL");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, VG_EDEVICE, "hipSetDevice failed");
  return tuple_neighbors(d, n_nodes, n_tuples, sigma, offsets, nbr, nbr_capacity, nnz, ctx->stream,
                         ctx->err);
}

}  // extern "C"

namespace {

int mc_backward(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                const float *dirs, uint64_t seed, bool seeded, const float *t, const int32_t *idx,
                const int32_t *facet_j, const int32_t *facet_count, const float *g_volume,
                const float *g_energy2, const float *g_facet_area, float *grad_nodes) {
  int rc = check_common(ctx, d, n_nodes, nodes);
  if (rc) return rc;
  if (rays_per_cell < 1 || rays_per_cell > 4096)
    return fail(ctx, VG_EINVAL, "rays_per_cell=%d outside [1, 4096]", rays_per_cell);
  if ((!dirs && !seeded) || !t || !idx || !grad_nodes) return fail(ctx, VG_EINVAL, "null array");
  if (seeded) dirs = nullptr;
  if (g_facet_area && (!facet_j || !facet_count))
    return fail(ctx, VG_EINVAL, "g_facet_area needs facet_j and facet_count");
  const int64_t n = n_nodes, m = n * (int64_t)rays_per_cell;
  size_t need = Carver::need({(size_t)n * d * 4, (size_t)m * d * 4, (size_t)m * 4, (size_t)n * 4,
                              (size_t)n * 4, (size_t)n * d * 8});
  rc = ensure_scratch(ctx, need);
  if (rc) return rc;
  Carver cv(ctx->scratch);
  BackwardArgs a{};
  a.own = cv.take<float>((size_t)n * d);
  a.rec = cv.take<float>((size_t)m * d);
  a.rec_j = cv.take<int32_t>((size_t)m);
  a.maxabs = cv.take<uint32_t>((size_t)n);
  a.count = cv.take<uint32_t>((size_t)n);
  a.acc = cv.take<unsigned long long>((size_t)n * d);
  VG_HIP(ctx, fill_u32(a.maxabs, 0u, n, ctx->stream));
  VG_HIP(ctx, fill_u32(a.count, 0u, n, ctx->stream));
  VG_HIP(ctx, fill_u32(reinterpret_cast<uint32_t *>(a.acc), 0u, 2 * n * d, ctx->stream));
  const double S = sphere_area(d);
  a.nodes = nodes;
  a.n = n;
  a.d = d;
  a.R = rays_per_cell;
  a.dirs = dirs;
  a.seed = seed;
  a.t = t;
  a.idx = idx;
  a.facet_j = facet_j;
  a.facet_count = facet_count;
  a.gv = g_volume;
  a.ge = g_energy2;
  a.ga = g_facet_area;
  a.sv = (float)(S / ((double)d * rays_per_cell));
  a.se = (float)(S / ((double)(d + 2) * rays_per_cell));
  a.sa = (float)(S / (double)rays_per_cell);
  a.grad = grad_nodes;
  hipError_t e = launch_backward(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "backward launch");
  return VG_OK;
}

}  // namespace

extern "C" {

int vg_mc_backward(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                   const float *dirs, const float *t, const int32_t *idx, const int32_t *facet_j,
                   const int32_t *facet_count, const float *g_volume, const float *g_energy2,
                   const float *g_facet_area, float *grad_nodes) {
  return mc_backward(ctx, d, n_nodes, nodes, rays_per_cell, dirs, 0, false, t, idx, facet_j, facet_count,
                     g_volume, g_energy2, g_facet_area, grad_nodes);
}

int vg_mc_backward_seeded(vg_ctx *ctx, int d, int64_t n_nodes, const float *nodes, int rays_per_cell,
                          uint64_t seed, const float *t, const int32_t *idx, const int32_t *facet_j,
                          const int32_t *facet_count, const float *g_volume, const float *g_energy2,
                          const float *g_facet_area, float *grad_nodes) {
  return mc_backward(ctx, d, n_nodes, nodes, rays_per_cell, nullptr, seed, true, t, idx, facet_j, facet_count,
                     g_volume, g_energy2, g_facet_area, grad_nodes);
}

}  // extern "C"
