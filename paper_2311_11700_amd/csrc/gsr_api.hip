// C ABI of the renderer: context, plan and workspace layout, the render
// entry points, HIP-graph capture of the fused step, and the autotuner.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gsr_internal.h"

using namespace gsr;

struct gsr_ctx {
  int device = 0;
  int num_cus = 256;
  Plan plan;
  bool planned = false;
  std::vector<ViewInfo> views_host;
  ViewInfo *views_dev = nullptr;
  int32_t *tile_view_dev = nullptr;
  unsigned long long *pinned = nullptr;  // 8 pinned host words
  std::string last_error;
  int64_t required = 0;
  Tuning tuning;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *last_forward_ws = nullptr;
  int64_t fwd_generation = 0;  // successful gsr_render_forward calls on this context
  void *scratch = nullptr;     // device address of this device's static scratch (gsr_render_l1_fused_noalloc)
  int sort_grid = 2048;
  // stage timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;   // (GSR_NSTAGES + 1) events per timed call
  size_t ev_used = 0;                // event sets recorded and not yet summed
  double stage_ms[GSR_NSTAGES] = {};
  int64_t timed_calls = 0;
  hipEvent_t *cur_events = nullptr;  // events of the call being enqueued
};

// Workspace of the allocation-free fused step (gsr_render_l1_fused_noalloc):
// a file-scope device array that every GPU the library runs on holds until
// the process ends.  In host code its name is not a device address; the
// address is taken once per device with hipGetSymbolAddress (gsr_create) and
// only that pointer is passed to kernels.
static __device__ __align__(256) unsigned char scratch[GSR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t ALIGN = 256;

// Per-device address of `scratch`, resolved on the first gsr_create on the
// device (with the device current).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

gsr_status fail(gsr_ctx *ctx, gsr_status st, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

gsr_status hip_check(gsr_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return GSR_OK;
  return fail(ctx, GSR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

gsr_status last_launch(gsr_ctx *ctx, const char *what) {
  return hip_check(ctx, hipGetLastError(), what);
}

int passes_for(int bits) { return (bits + RADIX_BITS - 1) / RADIX_BITS; }

Workspace make_ws(const Plan &p, void *base_v) {
  char *base = static_cast<char *>(base_v);
  Workspace w{};
  w.hdr = reinterpret_cast<uint32_t *>(base + p.off_hdr);
  w.recA = reinterpret_cast<float4 *>(base + p.off_recA);
  w.recB = reinterpret_cast<float4 *>(base + p.off_recB);
  w.recC = reinterpret_cast<float4 *>(base + p.off_recC);
  w.tinfo = reinterpret_cast<uint4 *>(base + p.off_rect);
  w.support = reinterpret_cast<Support *>(base + p.off_support);
  w.count = reinterpret_cast<uint32_t *>(base + p.off_count);
  w.tile_visible = reinterpret_cast<uint32_t *>(base + p.off_tile_visible);
  for (int k = 0; k < 2; ++k) {
    w.dkeys[k] = reinterpret_cast<uint32_t *>(base + p.off_dkeys[k]);
    w.dvals[k] = reinterpret_cast<uint32_t *>(base + p.off_dvals[k]);
    w.pkeys[k] = reinterpret_cast<uint32_t *>(base + p.off_pkeys[k]);
    w.pvals[k] = reinterpret_cast<uint32_t *>(base + p.off_pvals[k]);
  }
  w.hist = reinterpret_cast<uint32_t *>(base + p.off_hist);
  w.hoff = reinterpret_cast<uint32_t *>(base + p.off_hoff);
  w.bucket_rec = reinterpret_cast<uint32_t *>(base + p.off_bucket);
  w.digit_total = reinterpret_cast<uint32_t *>(base + p.off_digit);
  w.whist = reinterpret_cast<unsigned long long *>(base + p.off_whist);
  w.whoff = reinterpret_cast<unsigned long long *>(base + p.off_whoff);
  w.wdigit = reinterpret_cast<unsigned long long *>(base + p.off_wdigit);
  w.ranges = reinterpret_cast<int2 *>(base + p.off_ranges);
  w.T_final = reinterpret_cast<float *>(base + p.off_T);
  w.last = reinterpret_cast<int32_t *>(base + p.off_last);
  w.zr = reinterpret_cast<float *>(base + p.off_zr);
  w.counts = reinterpret_cast<unsigned long long *>(base + p.off_counts);
  w.grad2d = reinterpret_cast<double *>(base + p.off_grad2d);
  w.pose_part = reinterpret_cast<double *>(base + p.off_pose);
  w.queue = reinterpret_cast<uint32_t *>(base + p.off_queue);
  w.tile_cost = reinterpret_cast<uint32_t *>(base + p.off_tile_cost);
  w.expand_bits = reinterpret_cast<unsigned long long *>(base + p.off_expand_bits);
  w.expand_cnt = reinterpret_cast<uint32_t *>(base + p.off_expand_cnt);
  w.loss_part = reinterpret_cast<float *>(base + p.off_loss);
  w.dsorted = passes_for(32) & 1;
  w.psorted = passes_for(p.tile_bits) & 1;
  w.pack_shift = p.pack_shift;
  w.id_mask = p.pack_shift ? (1u << p.pack_shift) - 1u : 0xFFFFFFFFu;
  return w;
}

gsr_status validate(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                    const gsr_config *cfg, void *ws, size_t ws_bytes) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->planned) return fail(ctx, GSR_E_STATE, "gsr_plan() has not been called");
  if (!g || !cams || !cfg || !ws) return fail(ctx, GSR_E_INVALID, "null argument");
  if (g->n != ctx->plan.n) return fail(ctx, GSR_E_INVALID, "Gaussian count differs from the plan");
  if (n_views != ctx->plan.n_views) return fail(ctx, GSR_E_INVALID, "view count differs from the plan");
  if (ws_bytes < ctx->plan.bytes) return fail(ctx, GSR_E_INVALID, "workspace smaller than gsr_plan() requires");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN) return fail(ctx, GSR_E_INVALID, "workspace not 256-byte aligned");
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || (!g->rgb && !g->sh)))
    return fail(ctx, GSR_E_INVALID, "null Gaussian parameter array");
  if (reinterpret_cast<uintptr_t>(g->quat) % 16) return fail(ctx, GSR_E_INVALID, "quat must be 16-byte aligned");
  if (!(cfg->alpha_max > 0.f && cfg->alpha_max <= 1.f) || !(cfg->alpha_min >= 0.f && cfg->alpha_min <= 1.f) ||
      cfg->T_min < 0.f ||
      !(cfg->cutoff_sigma > 0.f) || !(cfg->fov_guard >= 0.f && cfg->fov_guard < 1e30f))
    return fail(ctx, GSR_E_INVALID, "renderer constants out of range");
  return GSR_OK;
}

RenderConsts consts(const gsr_config &c, const gsr_gaussians &g) {
  RenderConsts rc;
  rc.alpha_min = c.alpha_min;
  rc.alpha_max = c.alpha_max;
  rc.T_min = c.T_min;
  rc.bg[0] = c.bg[0];
  rc.bg[1] = c.bg[1];
  rc.bg[2] = c.bg[2];
  // Opacity and colour gradients (fields 5-8) feed only the Gaussian
  // parameters, except that spherical-harmonic colour depends on the
  // viewing direction and so on the pose; a pose-only backward skips the rest.
  rc.grad_fields = (c.flags & GSR_GAUSS_GRAD) ? 0x3FFu : (g.sh ? 0x3FFu & ~0x020u : 0x3FFu & ~0x1E0u);
  rc.id_mask = 0xFFFFFFFFu;
  return rc;
}

constexpr int NEV = GSR_NSTAGES + 1;

// Sum the recorded event sets into stage_ms (synchronises on the events).
gsr_status drain_events(gsr_ctx *ctx) {
  for (size_t k = 0; k < ctx->ev_used; ++k) {
    hipEvent_t *e = &ctx->ev_pool[k * NEV];
    gsr_status st = hip_check(ctx, hipEventSynchronize(e[NEV - 1]), "hipEventSynchronize");
    if (st != GSR_OK) return st;
    for (int j = 0; j < GSR_NSTAGES; ++j) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e[j], e[j + 1]) == hipSuccess) ctx->stage_ms[j] += ms;
    }
    ++ctx->timed_calls;
  }
  ctx->ev_used = 0;
  return GSR_OK;
}

// Start timing one call: take an event set (draining the pool when full).
void prof_begin(gsr_ctx *ctx, hipStream_t s) {
  ctx->cur_events = nullptr;
  if (!ctx->profiling) return;
  const size_t sets = ctx->ev_pool.size() / NEV;
  if (ctx->ev_used == sets) (void)drain_events(ctx);
  ctx->cur_events = &ctx->ev_pool[ctx->ev_used * NEV];
  ++ctx->ev_used;
  (void)hipEventRecord(ctx->cur_events[0], s);
}

// Mark the end of `stage` (stages run in enum order; skipped stages time ~0).
void prof_mark(gsr_ctx *ctx, hipStream_t s, int stage) {
  if (ctx->cur_events) (void)hipEventRecord(ctx->cur_events[stage + 1], s);
}

// Mark the end of every stage from `first_unmarked` on (the work enqueued
// since the last mark belongs to `first_unmarked`; later stages time ~0).
void prof_end(gsr_ctx *ctx, hipStream_t s, int first_unmarked) {
  if (!ctx->cur_events) return;
  for (int j = first_unmarked; j < GSR_NSTAGES; ++j) (void)hipEventRecord(ctx->cur_events[j + 1], s);
  ctx->cur_events = nullptr;
}

// Projection, depth sort, pair emission, tile sort and ranges.  The
// projection also resets the header, clears grad2d for a fused step, zeroes
// the fused step's loss when the gradients are overwritten and, with
// order_queue, writes the rasteriser's longest-first work order.
void enqueue_lists(gsr_ctx *ctx, const gsr_gaussians &g, const gsr_camera *cams, const gsr_config &cfg,
                   Workspace &ws, bool clear_grad2d, float *loss_zero, bool order_queue, hipStream_t s) {
  const Plan &p = ctx->plan;
  launch_preprocess(g, cams, ctx->views_dev, p.n_views, cfg, ws, clear_grad2d, loss_zero, p.max_sort_tiles,
                    order_queue ? p.total_tiles : 0, s);
  prof_mark(ctx, s, GSR_STAGE_PREPROCESS);
  launch_depth_sort(p, ws, s, ctx->sort_grid);
  prof_mark(ctx, s, GSR_STAGE_DEPTH_SORT);
  launch_emit_pairs(p, ws, ctx->views_dev, s);
  prof_mark(ctx, s, GSR_STAGE_EMIT);
  launch_pair_sort(p, ws, s, ctx->sort_grid);
  prof_mark(ctx, s, GSR_STAGE_PAIR_SORT);
  launch_tile_ranges(p, ws, s);
}

void enqueue_fused(gsr_ctx *ctx, const gsr_gaussians &g, const gsr_camera *cams, const gsr_config &cfg,
                   const float *t_rgb, const float *t_depth, const uint8_t *pmask, float w_rgb, float w_depth,
                   const float *loss_cap,
                   Workspace &ws, const gsr_images *out, const gsr_grads &gr, float *loss, hipStream_t s) {
  const Plan &p = ctx->plan;
  prof_begin(ctx, s);
  enqueue_lists(ctx, g, cams, cfg, ws, true, (cfg.flags & GSR_GRAD_OVERWRITE) ? loss : nullptr,
                ctx->tuning.lpt_order != 0, s);
  prof_mark(ctx, s, GSR_STAGE_RANGES);
  launch_render_fused(p, ws, ctx->views_dev, ctx->tile_view_dev, g, consts(cfg, g), t_rgb, t_depth, pmask, w_rgb,
                      w_depth, loss_cap, out, loss, ctx->tuning, ctx->num_cus, s);
  prof_mark(ctx, s, GSR_STAGE_RASTER);
  prof_mark(ctx, s, GSR_STAGE_RASTER_BWD);
  launch_preprocess_backward(p, g, cams, cfg, ws, gr, s);
  prof_end(ctx, s, GSR_STAGE_PREGRAD);
}

}  // namespace

static_assert(sizeof(gsr_camera) == 80, "gsr_camera layout");
static_assert(sizeof(gsr_config) == 44, "gsr_config layout");
static_assert(sizeof(gsr_gaussians_out) == 48, "gsr_gaussians_out layout");

extern "C" {

gsr_config gsr_default_config(void) {
  gsr_config c;
  c.alpha_min = 1.0f / 255.0f;
  c.alpha_max = 0.99f;
  c.T_min = 1e-4f;
  c.cutoff_sigma = 3.0f;
  c.z_near = 0.2f;
  c.lowpass = 0.3f;
  c.bg[0] = c.bg[1] = c.bg[2] = 0.f;
  c.flags = GSR_GAUSS_GRAD | GSR_POSE_GRAD;
  c.fov_guard = 1.3f;
  return c;
}

const char *gsr_status_string(gsr_status s) {
  switch (s) {
    case GSR_OK: return "GSR_OK";
    case GSR_E_INVALID: return "GSR_E_INVALID: invalid argument";
    case GSR_E_CAPACITY: return "GSR_E_CAPACITY: tile-pair buffer too small";
    case GSR_E_HIP: return "GSR_E_HIP: HIP runtime error";
    case GSR_E_UNSUPPORTED: return "GSR_E_UNSUPPORTED: unsupported configuration";
    case GSR_E_STATE: return "GSR_E_STATE: call out of order";
  }
  return "unknown gsr_status";
}

const char *gsr_last_error(const gsr_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

gsr_status gsr_create(int device, gsr_ctx **out) {
  if (!out) return GSR_E_INVALID;
  *out = nullptr;
  gsr_ctx *ctx = new gsr_ctx();
  ctx->device = device;
  gsr_status st = hip_check(ctx, hipSetDevice(device), "hipSetDevice");
  if (st == GSR_OK) st = hip_check(ctx, hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
  if (st == GSR_OK) st = hip_check(ctx, hipHostMalloc(reinterpret_cast<void **>(&ctx->pinned), 8 * sizeof(unsigned long long), hipHostMallocDefault), "hipHostMalloc");
  if (st == GSR_OK && device >= 0 && device < MAX_DEVICES) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void *ptr = nullptr;
      st = hip_check(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
      if (st == GSR_OK) g_scratch_ptr[device] = ptr;
    }
    ctx->scratch = g_scratch_ptr[device];
  }
  if (st != GSR_OK) {
    std::fprintf(stderr, "gsr_create: %s\n", ctx->last_error.c_str());
    gsr_destroy(ctx);
    return st;
  }
  *out = ctx;
  return GSR_OK;
}

void gsr_destroy(gsr_ctx *ctx) {
  if (!ctx) return;
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->views_dev) (void)hipFree(ctx->views_dev);
  if (ctx->tile_view_dev) (void)hipFree(ctx->tile_view_dev);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

gsr_status gsr_plan(gsr_ctx *ctx, int64_t n, int n_views, const int32_t *wh_host, int64_t pair_capacity,
                    size_t *workspace_bytes) {
  if (!ctx) return GSR_E_INVALID;
  if (n < 0 || n_views < 1 || !wh_host || pair_capacity < 1 || !workspace_bytes)
    return fail(ctx, GSR_E_INVALID, "gsr_plan: invalid argument");
  if (n_views > 256) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_plan: at most 256 views per call");
  if (pair_capacity >= (int64_t)0xFFFFFFFFll) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_plan: pair capacity must be < 2^32 - 1");
  if (n * (int64_t)n_views >= (int64_t)0xFFFFFFFFll) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_plan: n * n_views must be < 2^32 - 1");
  Plan p;
  p.n = n;
  p.n_views = n_views;
  p.n_rec = n * n_views;
  p.capacity = pair_capacity;
  std::vector<ViewInfo> views(n_views);
  int64_t tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = wh_host[2 * v], H = wh_host[2 * v + 1];
    if (W < 1 || H < 1) return fail(ctx, GSR_E_INVALID, "gsr_plan: view size must be positive");
    if (W > 65535 || H > 65535) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_plan: view larger than 65535 px");
    ViewInfo &vi = views[v];
    vi.W = W;
    vi.H = H;
    vi.TX = (W + TILE - 1) / TILE;
    vi.TY = (H + TILE - 1) / TILE;
    vi.tile_off = (int32_t)tiles;
    vi._pad = 0;
    vi.pix_off = pixels;
    tiles += (int64_t)vi.TX * vi.TY;
    pixels += (int64_t)W * H;
  }
  if (tiles >= (1ll << 31)) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_plan: too many tiles");
  p.total_tiles = (int)tiles;
  p.total_pixels = pixels;
  // Tile keys 0..tiles-1 plus one key past the last tile for the pairs
  // outside a Gaussian's alpha support.
  int bits = 0;
  while ((1ll << bits) < tiles + 1) ++bits;
  p.tile_bits = bits;
  int rbits = 1;
  while ((1ll << rbits) < p.n_rec) ++rbits;
  p.pack_shift = bits + rbits <= 32 ? rbits : 0;
  const int64_t dtile = (int64_t)BLOCK * SORT_ITEMS_DEPTH, ptile = (int64_t)BLOCK * SORT_ITEMS_PAIR;
  p.max_sort_tiles = (int)std::max<int64_t>((p.n_rec + dtile - 1) / dtile, (p.capacity + ptile - 1) / ptile);
  p.depth_tiles = (int)std::max<int64_t>(1, (p.n_rec + dtile - 1) / dtile);
  p.n_pose_blocks = (int)std::max<int64_t>(1, (n + BLOCK - 1) / BLOCK);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t nr = (size_t)p.n_rec, cap = (size_t)p.capacity;
  p.off_hdr = take(HDR_WORDS * 4);
  p.off_recA = take(16 * nr);
  p.off_recB = take(16 * nr);
  p.off_recC = take(16 * nr);
  p.off_rect = take(16 * nr);
  p.off_support = take(sizeof(Support) * nr);
  p.off_count = take(4 * nr);
  p.off_tile_visible = take(4 * (size_t)((nr + (size_t)BLOCK * SORT_ITEMS_DEPTH - 1) / ((size_t)BLOCK * SORT_ITEMS_DEPTH)));
  for (int k = 0; k < 2; ++k) p.off_dkeys[k] = take(4 * nr);
  for (int k = 0; k < 2; ++k) p.off_dvals[k] = take(4 * nr);
  for (int k = 0; k < 2; ++k) p.off_pkeys[k] = take(4 * cap);
  for (int k = 0; k < 2; ++k) p.off_pvals[k] = take(4 * cap);
  p.off_hist = take(4 * (size_t)RADIX * p.max_sort_tiles);
  p.off_hoff = take(4 * (size_t)RADIX * p.max_sort_tiles);
  p.off_bucket = take(4 * (cap / EMIT_BUCKET + 2));
  p.off_digit = take(4 * RADIX);
  p.off_whist = take(8 * (size_t)RADIX * p.depth_tiles);
  p.off_whoff = take(8 * (size_t)RADIX * p.depth_tiles);
  p.off_wdigit = take(8 * RADIX);
  p.off_ranges = take(8 * (size_t)p.total_tiles);
  p.off_T = take(4 * (size_t)pixels);
  p.off_last = take(4 * (size_t)pixels);
  p.off_zr = take(4 * (size_t)pixels);
  p.off_counts = take(64);
  p.off_grad2d = take(8 * NGRAD2D * nr);
  p.off_pose = take(8 * 6 * (size_t)n_views * p.n_pose_blocks);
  p.off_queue = take(4 * (size_t)p.total_tiles);
  p.off_tile_cost = take(4 * (size_t)p.total_tiles);
  p.off_loss = take(4);
  {
    const size_t chunks = (size_t)((pixels + EXPAND_CHUNK - 1) / EXPAND_CHUNK);
    p.off_expand_bits = take(8 * chunks * (EXPAND_CHUNK / 64));
    p.off_expand_cnt = take(4 * chunks);
  }
  p.bytes = off;

  gsr_status st = hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (st != GSR_OK) return st;
  if (ctx->views_dev) (void)hipFree(ctx->views_dev);
  if (ctx->tile_view_dev) (void)hipFree(ctx->tile_view_dev);
  ctx->views_dev = nullptr;
  ctx->tile_view_dev = nullptr;
  ctx->planned = false;
  std::vector<int32_t> tv(tiles);
  for (int v = 0; v < n_views; ++v)
    for (int64_t t = 0; t < (int64_t)views[v].TX * views[v].TY; ++t) tv[views[v].tile_off + t] = v;
  st = hip_check(ctx, hipMalloc(reinterpret_cast<void **>(&ctx->views_dev), sizeof(ViewInfo) * n_views), "hipMalloc(views)");
  if (st == GSR_OK) st = hip_check(ctx, hipMalloc(reinterpret_cast<void **>(&ctx->tile_view_dev), sizeof(int32_t) * tiles), "hipMalloc(tile_view)");
  if (st == GSR_OK) st = hip_check(ctx, hipMemcpy(ctx->views_dev, views.data(), sizeof(ViewInfo) * n_views, hipMemcpyHostToDevice), "hipMemcpy(views)");
  if (st == GSR_OK) st = hip_check(ctx, hipMemcpy(ctx->tile_view_dev, tv.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice), "hipMemcpy(tile_view)");
  if (st != GSR_OK) return st;
  ctx->plan = p;
  ctx->views_host = views;
  ctx->planned = true;
  ctx->last_forward_ws = nullptr;
  *workspace_bytes = p.bytes;
  return GSR_OK;
}

gsr_status gsr_render_forward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                              const gsr_config *cfg, void *workspace, size_t workspace_bytes,
                              const gsr_images *out, gsr_stream stream) {
  gsr_status st = validate(ctx, g, cams, n_views, cfg, workspace, workspace_bytes);
  if (st != GSR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  prof_begin(ctx, s);
  enqueue_lists(ctx, *g, cams, *cfg, ws, false, nullptr, false, s);
  prof_mark(ctx, s, GSR_STAGE_RANGES);
  launch_render_forward(ctx->plan, ws, ctx->views_dev, ctx->tile_view_dev, *g, consts(*cfg, *g), out, s);
  prof_end(ctx, s, GSR_STAGE_RASTER);
  if ((st = last_launch(ctx, "gsr_render_forward launch")) != GSR_OK) return st;
  ctx->last_forward_ws = workspace;
  ++ctx->fwd_generation;
  return GSR_OK;
}

int64_t gsr_forward_generation(const gsr_ctx *ctx) { return ctx ? ctx->fwd_generation : 0; }

gsr_status gsr_render_backward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                               const gsr_config *cfg, void *workspace, size_t workspace_bytes,
                               int64_t forward_generation, const float *g_rgb, const float *g_depth,
                               const float *g_T, const gsr_grads *grads, gsr_stream stream) {
  gsr_status st = validate(ctx, g, cams, n_views, cfg, workspace, workspace_bytes);
  if (st != GSR_OK) return st;
  if (!g_rgb || !grads) return fail(ctx, GSR_E_INVALID, "gsr_render_backward: null gradient argument");
  if (ctx->last_forward_ws != workspace)
    return fail(ctx, GSR_E_STATE, "gsr_render_backward: workspace was not filled by the last forward");
  if (forward_generation != ctx->fwd_generation)
    return fail(ctx, GSR_E_STATE, "gsr_render_backward: the workspace holds forward " +
                                      std::to_string(ctx->fwd_generation) + ", not forward " +
                                      std::to_string(forward_generation));
  if ((cfg->flags & GSR_GAUSS_GRAD) && g->n > 0 &&
      (!grads->d_mean || !grads->d_log_scale || !grads->d_quat || !grads->d_opacity_logit ||
       (g->sh ? !grads->d_sh : !grads->d_rgb)))
    return fail(ctx, GSR_E_INVALID, "GSR_GAUSS_GRAD needs every d_* pointer (d_sh instead of d_rgb with spherical-harmonic colour)");
  if ((cfg->flags & GSR_POSE_GRAD) && !grads->d_pose) return fail(ctx, GSR_E_INVALID, "GSR_POSE_GRAD needs d_pose");
  if (grads->d_quat && reinterpret_cast<uintptr_t>(grads->d_quat) % 16)
    return fail(ctx, GSR_E_INVALID, "d_quat must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  const Plan &p = ctx->plan;
  prof_begin(ctx, s);
  // The gradient rows are cleared inside the (otherwise empty) stages before
  // the backward rasteriser, so its stage times the kernel alone.
  launch_fill_f32(reinterpret_cast<float *>(ws.grad2d), 0.f, 2 * p.n_rec * NGRAD2D, s);
  for (int j = 0; j <= GSR_STAGE_RASTER; ++j) prof_mark(ctx, s, j);
  launch_render_backward(p, ws, ctx->views_dev, ctx->tile_view_dev, *g, consts(*cfg, *g), g_rgb, g_depth, g_T, s);
  prof_mark(ctx, s, GSR_STAGE_RASTER_BWD);
  launch_preprocess_backward(p, *g, cams, *cfg, ws, *grads, s);
  prof_end(ctx, s, GSR_STAGE_PREGRAD);
  return last_launch(ctx, "gsr_render_backward launch");
}

gsr_status gsr_l1_loss_grad(gsr_ctx *ctx, const float *rgb, const float *depth, const float *target_rgb,
                            const float *target_depth, const uint8_t *pixel_mask, float w_rgb, float w_depth,
                            const float *loss_cap, float *g_rgb, float *g_depth, float *loss, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->planned) return fail(ctx, GSR_E_STATE, "gsr_plan() has not been called");
  if (!rgb || !depth || !target_rgb || !target_depth || !g_rgb || !g_depth)
    return fail(ctx, GSR_E_INVALID, "gsr_l1_loss_grad: null argument");
  if (!(w_rgb >= 0.f) || !(w_depth >= 0.f)) return fail(ctx, GSR_E_INVALID, "loss weights must be >= 0");
  launch_l1(ctx->plan, ctx->views_dev, rgb, depth, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, loss_cap,
            g_rgb, g_depth, loss, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_l1_loss_grad launch");
}

gsr_status gsr_loss_median(gsr_ctx *ctx, const float *px_loss, const uint8_t *pixel_mask, float factor,
                           float *cap_out, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->planned) return fail(ctx, GSR_E_STATE, "gsr_plan() has not been called");
  if (!px_loss || !cap_out) return fail(ctx, GSR_E_INVALID, "gsr_loss_median: null argument");
  if (!(factor >= 0.f)) return fail(ctx, GSR_E_INVALID, "gsr_loss_median: factor must be >= 0");
  launch_loss_median(ctx->plan, ctx->views_dev, px_loss, pixel_mask, factor, cap_out,
                     static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_loss_median launch");
}

static gsr_status fused_checks(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                               const gsr_config *cfg, const float *t_rgb, const float *t_depth, float w_rgb,
                               float w_depth, void *ws, size_t ws_bytes, const gsr_grads *grads) {
  gsr_status st = validate(ctx, g, cams, n_views, cfg, ws, ws_bytes);
  if (st != GSR_OK) return st;
  if (!t_rgb || !t_depth || !grads) return fail(ctx, GSR_E_INVALID, "fused step: null target or gradient argument");
  if (!(w_rgb >= 0.f) || !(w_depth >= 0.f)) return fail(ctx, GSR_E_INVALID, "loss weights must be >= 0");
  if ((cfg->flags & GSR_GAUSS_GRAD) && g->n > 0 &&
      (!grads->d_mean || !grads->d_log_scale || !grads->d_quat || !grads->d_opacity_logit ||
       (g->sh ? !grads->d_sh : !grads->d_rgb)))
    return fail(ctx, GSR_E_INVALID, "GSR_GAUSS_GRAD needs every d_* pointer (d_sh instead of d_rgb with spherical-harmonic colour)");
  if ((cfg->flags & GSR_POSE_GRAD) && !grads->d_pose) return fail(ctx, GSR_E_INVALID, "GSR_POSE_GRAD needs d_pose");
  if (grads->d_quat && reinterpret_cast<uintptr_t>(grads->d_quat) % 16)
    return fail(ctx, GSR_E_INVALID, "d_quat must be 16-byte aligned");
  return GSR_OK;
}

gsr_status gsr_render_l1_fused(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                               const gsr_config *cfg, const float *target_rgb, const float *target_depth,
                               const uint8_t *pixel_mask, float w_rgb, float w_depth, const float *loss_cap,
                               void *workspace, size_t workspace_bytes, const gsr_images *out,
                               const gsr_grads *grads, float *loss, gsr_stream stream) {
  gsr_status st = fused_checks(ctx, g, cams, n_views, cfg, target_rgb, target_depth, w_rgb, w_depth, workspace,
                               workspace_bytes, grads);
  if (st != GSR_OK) return st;
  Workspace ws = make_ws(ctx->plan, workspace);
  enqueue_fused(ctx, *g, cams, *cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, loss_cap, ws, out,
                *grads, loss, static_cast<hipStream_t>(stream));
  ctx->last_forward_ws = nullptr;
  return last_launch(ctx, "gsr_render_l1_fused launch");
}

gsr_status gsr_render_l1_fused_noalloc(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                                       const gsr_config *cfg, const float *target_rgb, const float *target_depth,
                                       const uint8_t *pixel_mask, float w_rgb, float w_depth, const float *loss_cap,
                                       const gsr_images *out, const gsr_grads *grads, float *loss,
                                       gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->scratch) return fail(ctx, GSR_E_STATE, "gsr_render_l1_fused_noalloc: no static scratch on this device");
  if (!ctx->planned) return fail(ctx, GSR_E_STATE, "gsr_plan() has not been called");
  if (ctx->plan.bytes > GSR_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, GSR_E_INVALID, "gsr_render_l1_fused_noalloc: the plan needs " + std::to_string(ctx->plan.bytes) +
                                        " workspace bytes, the static scratch holds " +
                                        std::to_string((size_t)GSR_NOALLOC_SCRATCH_BYTES) +
                                        " (use gsr_render_l1_fused with a workspace)");
  gsr_status st = fused_checks(ctx, g, cams, n_views, cfg, target_rgb, target_depth, w_rgb, w_depth, ctx->scratch,
                               GSR_NOALLOC_SCRATCH_BYTES, grads);
  if (st != GSR_OK) return st;
  Workspace ws = make_ws(ctx->plan, ctx->scratch);
  enqueue_fused(ctx, *g, cams, *cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, loss_cap, ws, out,
                *grads, loss, static_cast<hipStream_t>(stream));
  ctx->last_forward_ws = nullptr;
  return last_launch(ctx, "gsr_render_l1_fused_noalloc launch");
}

gsr_status gsr_graph_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                             const gsr_config *cfg, const float *target_rgb, const float *target_depth,
                             const uint8_t *pixel_mask, float w_rgb, float w_depth, const float *loss_cap,
                             void *workspace, size_t workspace_bytes, const gsr_images *out,
                             const gsr_grads *grads, float *loss, gsr_stream stream) {
  gsr_status st = fused_checks(ctx, g, cams, n_views, cfg, target_rgb, target_depth, w_rgb, w_depth, workspace,
                               workspace_bytes, grads);
  if (st != GSR_OK) return st;
  if (!stream) return fail(ctx, GSR_E_INVALID, "gsr_graph_capture needs a non-null stream");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->gexec = nullptr;
  ctx->graph = nullptr;
  st = hip_check(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st != GSR_OK) return st;
  Workspace ws = make_ws(ctx->plan, workspace);
  const bool prof = ctx->profiling;
  ctx->profiling = false;  // no event records inside a captured graph
  enqueue_fused(ctx, *g, cams, *cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, loss_cap, ws, out,
                *grads, loss, s);
  ctx->profiling = prof;
  hipGraph_t graph = nullptr;
  st = hip_check(ctx, hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
  if (st != GSR_OK) return st;
  hipGraphExec_t exec = nullptr;
  st = hip_check(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (st != GSR_OK) {
    (void)hipGraphDestroy(graph);
    return st;
  }
  ctx->graph = graph;
  ctx->gexec = exec;
  ctx->last_forward_ws = nullptr;
  return GSR_OK;
}

gsr_status gsr_graph_launch(gsr_ctx *ctx, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->gexec) return fail(ctx, GSR_E_STATE, "no captured graph");
  return hip_check(ctx, hipGraphLaunch(ctx->gexec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

gsr_status gsr_check_overflow(gsr_ctx *ctx, void *workspace, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!workspace) workspace = ctx->scratch;  // the allocation-free step's static workspace
  if (!ctx->planned || !workspace) return fail(ctx, GSR_E_STATE, "gsr_check_overflow: no plan or workspace");
  if (workspace == ctx->scratch && ctx->plan.bytes > GSR_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, GSR_E_STATE, "gsr_check_overflow: the plan does not fit the static scratch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  gsr_status st = hip_check(ctx, hipMemcpyAsync(ctx->pinned, ws.hdr, 40, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (st == GSR_OK) st = hip_check(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
  if (st != GSR_OK) return st;
  const uint32_t flag = static_cast<uint32_t>(ctx->pinned[2] & 0xFFFFFFFFull);
  const bool used = ctx->pinned[4] == ((unsigned long long)HDR_MAGIC1 << 32 | HDR_MAGIC0);
  if (used && flag) {
    ctx->required = (int64_t)ctx->pinned[1];
    launch_fill_u32(ws.hdr + HDR_REQUIRED, 0u, 3, s);
    st = hip_check(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != GSR_OK) return st;
    return fail(ctx, GSR_E_CAPACITY, "pair buffer too small: need " + std::to_string(ctx->required));
  }
  return GSR_OK;
}

int64_t gsr_required_pairs(const gsr_ctx *ctx) { return ctx ? ctx->required : 0; }

int64_t gsr_pair_count(gsr_ctx *ctx, void *workspace, gsr_stream stream) {
  if (!ctx || !ctx->planned || !workspace) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  if (hipMemcpyAsync(ctx->pinned, ws.hdr + HDR_NPAIRS, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return (int64_t)ctx->pinned[0];
}

gsr_status gsr_debug_tiles(gsr_ctx *ctx, void *workspace, const int32_t **tile_ranges, const uint32_t **sorted_ids,
                           int64_t *total_tiles) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->planned || !workspace) return fail(ctx, GSR_E_STATE, "gsr_debug_tiles: no plan or workspace");
  Workspace ws = make_ws(ctx->plan, workspace);
  if (tile_ranges) *tile_ranges = reinterpret_cast<const int32_t *>(ws.ranges);
  if (sorted_ids) {
    if (ws.pack_shift) {
      // Packed words: write the record ids into the (unused) value buffer.
      gsr_status st = hip_check(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st != GSR_OK) return st;
      launch_unpack_ids(ctx->plan, ws, nullptr);
      st = hip_check(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st != GSR_OK) return st;
    }
    *sorted_ids = ws.pvals[ws.psorted];
  }
  if (total_tiles) *total_tiles = ctx->plan.total_tiles;
  return GSR_OK;
}

gsr_status gsr_get_tuning(const gsr_ctx *ctx, gsr_tuning *out) {
  if (!ctx || !out) return GSR_E_INVALID;
  out->blocks_per_cu = ctx->tuning.blocks_per_cu;
  out->tiles_per_pop = ctx->tuning.tiles_per_pop;
  out->lpt_order = ctx->tuning.lpt_order;
  out->batch = ctx->tuning.batch;
  return GSR_OK;
}

gsr_status gsr_set_tuning(gsr_ctx *ctx, const gsr_tuning *t) {
  if (!ctx || !t) return GSR_E_INVALID;
  const int batch = t->batch == 0 ? 192 : t->batch;
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 8 || t->tiles_per_pop < 1 || t->tiles_per_pop > 8 ||
      (batch != 64 && batch != 128 && batch != 192 && batch != 256))
    return fail(ctx, GSR_E_INVALID, "tuning out of range");
  ctx->tuning.blocks_per_cu = t->blocks_per_cu;
  ctx->tuning.tiles_per_pop = t->tiles_per_pop;
  ctx->tuning.lpt_order = t->lpt_order ? 1 : 0;
  ctx->tuning.batch = batch;
  return GSR_OK;
}

gsr_status gsr_autotune(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                        const gsr_config *cfg, const float *target_rgb, const float *target_depth,
                        const uint8_t *pixel_mask, float w_rgb, float w_depth, void *workspace,
                        size_t workspace_bytes, const gsr_grads *grads, float *loss, int reps, gsr_tuning *best,
                        gsr_stream stream) {
  gsr_status st = fused_checks(ctx, g, cams, n_views, cfg, target_rgb, target_depth, w_rgb, w_depth, workspace,
                               workspace_bytes, grads);
  if (st != GSR_OK) return st;
  if (reps < 1) reps = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  const Plan &p = ctx->plan;
  enqueue_lists(ctx, *g, cams, *cfg, ws, false, nullptr, false, s);
  hipEvent_t e0, e1;
  if ((st = hip_check(ctx, hipEventCreate(&e0), "hipEventCreate")) != GSR_OK) return st;
  if ((st = hip_check(ctx, hipEventCreate(&e1), "hipEventCreate")) != GSR_OK) {
    (void)hipEventDestroy(e0);
    return st;
  }
  const Tuning saved = ctx->tuning;
  Tuning best_t = saved;
  float best_ms = 1e30f;
  // Mean time of `reps` launches of the rasteriser alone (after one warm-up)
  // on the lists built above; keeps the fastest tuning.
  auto trial = [&](const Tuning &t, float margin) {
    float total = 0.f;
    for (int r = 0; r <= reps && st == GSR_OK; ++r) {
      launch_fill_u32(ws.hdr + HDR_QUEUE, 0u, 1, s);
      if (t.lpt_order) launch_queue_order(ws, p.total_tiles, s);
      launch_fill_f32(reinterpret_cast<float *>(ws.grad2d), 0.f, 2 * p.n_rec * NGRAD2D, s);
      (void)hipEventRecord(e0, s);
      launch_render_fused(p, ws, ctx->views_dev, ctx->tile_view_dev, *g, consts(*cfg, *g), target_rgb, target_depth,
                          pixel_mask, w_rgb, w_depth, nullptr, nullptr, loss, t, ctx->num_cus, s);
      (void)hipEventRecord(e1, s);
      st = hip_check(ctx, hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) total += ms;  // first run is a warm-up
    }
    if (st == GSR_OK && total / reps < best_ms * margin) {
      best_ms = total / reps;
      best_t = t;
    }
  };
  // Work order, blocks per CU and tiles per pop at the default batch, then
  // the other batch sizes at the best of those (taken only when 2 % faster,
  // so that timing noise does not flip the kernel).
  const int bpcs[] = {1, 2, 3, 4, 6, 8};
  const int pops[] = {1, 2, 4};
  for (int lpt = 0; lpt <= 1 && st == GSR_OK; ++lpt)
    for (int bpc : bpcs)
      for (int pop : pops) {
        Tuning t;
        t.blocks_per_cu = bpc;
        t.tiles_per_pop = pop;
        t.lpt_order = lpt;
        trial(t, 1.f);
      }
  const Tuning grid_best = best_t;
  for (int batch : {64, 128, 256}) {
    if (st != GSR_OK) break;
    Tuning t = grid_best;
    t.batch = batch;
    trial(t, 0.98f);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GSR_OK) return st;
  ctx->tuning = best_t;
  if (best) (void)gsr_get_tuning(ctx, best);
  ctx->last_forward_ws = nullptr;
  return last_launch(ctx, "gsr_autotune");
}

gsr_status gsr_select_reliable(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam,
                               const float *depth_obs, int width, int height, float eps, float z_near,
                               uint8_t *mask_out, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!g || !cam || !depth_obs || !mask_out || width < 1 || height < 1 || !(eps >= 0.f))
    return fail(ctx, GSR_E_INVALID, "gsr_select_reliable: invalid argument");
  if (g->n > 0 && !g->mean) return fail(ctx, GSR_E_INVALID, "gsr_select_reliable: null mean");
  launch_select_reliable(*g, cam, depth_obs, width, height, eps, z_near, mask_out, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_select_reliable launch");
}

gsr_status gsr_expand_add(gsr_ctx *ctx, const gsr_camera *cams, int n_views, const float *T_final, const float *depth,
                          const float *depth_obs, const float *rgb_obs, const gsr_expand_params *prm,
                          void *workspace, size_t workspace_bytes, int64_t n, int64_t capacity,
                          const gsr_gaussians_out *out, uint8_t *pixel_flag, int64_t *count, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!ctx->planned) return fail(ctx, GSR_E_STATE, "gsr_plan() has not been called");
  if (n_views != ctx->plan.n_views) return fail(ctx, GSR_E_INVALID, "gsr_expand_add: view count differs from the plan");
  if (!cams || !T_final || !depth || !depth_obs || !rgb_obs || !prm || !workspace || !count)
    return fail(ctx, GSR_E_INVALID, "gsr_expand_add: null argument");
  if (workspace_bytes < ctx->plan.bytes) return fail(ctx, GSR_E_INVALID, "workspace smaller than gsr_plan() requires");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return fail(ctx, GSR_E_INVALID, "workspace not 256-byte aligned");
  if (n < 0 || capacity < n) return fail(ctx, GSR_E_INVALID, "gsr_expand_add: need 0 <= n <= capacity");
  if (capacity > n && (!out || !out->mean || !out->log_scale || !out->quat || !out->opacity_logit ||
                       (!out->rgb && !out->sh)))
    return fail(ctx, GSR_E_INVALID, "gsr_expand_add: null output array");
  if (out && reinterpret_cast<uintptr_t>(out->quat) % 16) return fail(ctx, GSR_E_INVALID, "quat must be 16-byte aligned");
  if (!(prm->tau_T >= 0.f && prm->tau_T < 1e30f) || !(prm->tau_D >= 0.f && prm->tau_D < 1e30f) ||
      !(prm->scale_factor > 0.f && prm->scale_factor < 1e30f) || !(fabsf(prm->opacity_logit_init) < 1e30f))
    return fail(ctx, GSR_E_INVALID, "gsr_expand_add: parameters out of range");
  gsr_gaussians_out o{};
  if (out) o = *out;
  launch_expand_add(ctx->plan, ctx->views_dev, cams, T_final, depth, depth_obs, rgb_obs, prm->tau_T, prm->tau_D,
                    prm->scale_factor, prm->opacity_logit_init, make_ws(ctx->plan, workspace), n, capacity, o,
                    pixel_flag, count, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_expand_add launch");
}

gsr_status gsr_expand_delete(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam, const float *depth_obs,
                             int width, int height, float gamma, float eta, float z_near, float *opacity_logit_out,
                             uint8_t *decayed, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (!g || !cam || !depth_obs || width < 1 || height < 1 || !(gamma >= 0.f && gamma < 1e30f) ||
      !(eta > 0.f && eta <= 1.f) || !(z_near >= 0.f))
    return fail(ctx, GSR_E_INVALID, "gsr_expand_delete: invalid argument");
  if (g->n > 0 && (!g->mean || !g->opacity_logit || !opacity_logit_out))
    return fail(ctx, GSR_E_INVALID, "gsr_expand_delete: null array");
  launch_expand_delete(*g, cam, depth_obs, width, height, gamma, eta, z_near, opacity_logit_out, decayed,
                       static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_expand_delete launch");
}

gsr_status gsr_pose_apply(gsr_ctx *ctx, int n_views, const float *xi, const gsr_camera *cams_in,
                          gsr_camera *cams_out, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (n_views < 0 || (n_views > 0 && (!xi || !cams_in || !cams_out)))
    return fail(ctx, GSR_E_INVALID, "gsr_pose_apply: invalid argument");
  launch_pose_apply(n_views, xi, cams_in, cams_out, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_pose_apply launch");
}

gsr_status gsr_pose_xi_grad(gsr_ctx *ctx, int n_views, const float *xi, const float *d_pose, float *d_xi,
                            gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (n_views < 0 || (n_views > 0 && (!xi || !d_pose || !d_xi)))
    return fail(ctx, GSR_E_INVALID, "gsr_pose_xi_grad: invalid argument");
  launch_pose_xi_grad(n_views, xi, d_pose, d_xi, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_pose_xi_grad launch");
}

gsr_status gsr_pose_from_qt(gsr_ctx *ctx, int n_views, const float *q, const float *t, const gsr_camera *cams_in,
                            gsr_camera *cams_out, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (n_views < 0 || (n_views > 0 && (!q || !t || !cams_in || !cams_out)))
    return fail(ctx, GSR_E_INVALID, "gsr_pose_from_qt: invalid argument");
  launch_pose_from_qt(n_views, q, t, cams_in, cams_out, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_pose_from_qt launch");
}

gsr_status gsr_pose_qt_grad(gsr_ctx *ctx, int n_views, const float *q, const float *t, const float *d_pose,
                            float *d_q, float *d_t, gsr_stream stream) {
  if (!ctx) return GSR_E_INVALID;
  if (n_views < 0 || (n_views > 0 && (!q || !t || !d_pose || !d_q || !d_t)))
    return fail(ctx, GSR_E_INVALID, "gsr_pose_qt_grad: invalid argument");
  launch_pose_qt_grad(n_views, q, t, d_pose, d_q, d_t, static_cast<hipStream_t>(stream));
  return last_launch(ctx, "gsr_pose_qt_grad launch");
}

gsr_status gsr_set_profiling(gsr_ctx *ctx, int enable) {
  if (!ctx) return GSR_E_INVALID;
  if (enable && ctx->ev_pool.empty()) {
    ctx->ev_pool.resize((size_t)NEV * 64);
    for (auto &e : ctx->ev_pool) {
      gsr_status st = hip_check(ctx, hipEventCreate(&e), "hipEventCreate");
      if (st != GSR_OK) return st;
    }
  }
  ctx->profiling = enable != 0;
  return GSR_OK;
}

gsr_status gsr_stage_times(gsr_ctx *ctx, double *ms, int64_t *calls) {
  if (!ctx || !ms) return GSR_E_INVALID;
  gsr_status st = drain_events(ctx);
  if (st != GSR_OK) return st;
  for (int j = 0; j < GSR_NSTAGES; ++j) {
    ms[j] = ctx->stage_ms[j];
    ctx->stage_ms[j] = 0.0;
  }
  if (calls) *calls = ctx->timed_calls;
  ctx->timed_calls = 0;
  return GSR_OK;
}

gsr_status gsr_work_counts(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_config *cfg, void *workspace,
                           gsr_stream stream, int64_t *out) {
  if (!ctx || !out || !g || !cfg) return GSR_E_INVALID;
  if (!ctx->planned || !workspace) return fail(ctx, GSR_E_STATE, "gsr_work_counts: no plan or workspace");
  if (g->n != ctx->plan.n) return fail(ctx, GSR_E_INVALID, "Gaussian count differs from the plan");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws = make_ws(ctx->plan, workspace);
  launch_work_counts(ctx->plan, ws, ctx->views_dev, ctx->tile_view_dev, *g, consts(*cfg, *g), s);
  unsigned long long host[4];
  gsr_status st = hip_check(ctx, hipMemcpyAsync(host, ws.counts, sizeof(host), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (st == GSR_OK) st = hip_check(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
  if (st != GSR_OK) return st;
  for (int k = 0; k < 4; ++k) out[k] = (int64_t)host[k];
  return GSR_OK;
}

}  // extern "C"
