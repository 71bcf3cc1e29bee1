// Internal declarations of the gfx950 splatting renderer: the view table,
// the workspace layout, device helpers shared by the kernels, and the kernel
// launchers the C ABI calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

constexpr int TILE = 16;          // tile edge in pixels
constexpr int BLOCK = 256;        // one thread per pixel of a tile
constexpr int NGRAD2D = 10;       // u, v, conic a, b, c, opacity, r, g, b, depth
constexpr int SORT_ITEMS_DEPTH = 2;  // keys per thread per sort tile, depth sort of the records
constexpr int SORT_ITEMS_PAIR = 8;  // keys per thread per sort tile, tile sort of the pairs
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SCAN_ITEMS = 8;
constexpr int EMIT_BUCKET = 256;  // pairs per emission bucket (one block-iteration of k_emit_pairs)
constexpr int EXPAND_CHUNK = 2048;  // pixels per block of the adding step (eight rounds of BLOCK)
// Real spherical harmonics of degree <= 1: 1/(2 sqrt(pi)) and sqrt(3/(4 pi)).
constexpr double SH_C0 = 0.28209479177387814;
constexpr double SH_C1 = 0.48860251190291992;

// Bits per radix pass for keys of key_bits bits: ceil(key_bits / 8) passes
// with the bits spread evenly (fewer digit values make longer output runs).
__host__ __device__ constexpr int radix_digit_bits(int key_bits) {
  return (key_bits + (key_bits + RADIX_BITS - 1) / RADIX_BITS - 1) / ((key_bits + RADIX_BITS - 1) / RADIX_BITS);
}

// Per-view geometry of the concatenated output (device copy lives in the
// context, written at plan time).
struct ViewInfo {
  int32_t W, H, TX, TY;
  int32_t tile_off;   // first global tile id of the view
  int32_t _pad;
  int64_t pix_off;    // first pixel of the view in the concatenated images
};

// Header words at the start of the workspace.
enum HeaderWord {
  HDR_NPAIRS = 0,      // u64 (words 0-1): pairs produced by the last forward
  HDR_REQUIRED = 2,    // u64 (words 2-3): largest pair count seen that overflowed
  HDR_OVERFLOW = 4,    // u32: set when a forward overflowed the pair buffer
  HDR_QUEUE = 5,       // u32: persistent rasteriser work counter
  HDR_FWD_DONE = 6,    // u32: marker that a forward filled this workspace
  HDR_MAGIC = 8,       // u32 x 2 (words 8-9): set once the header has been initialised
  HDR_NVISIBLE = 10,   // u64 (words 10-11): records that passed the culling (depth-sorted keys)
  HDR_NLISTED = 12,    // u64 (words 12-13): pairs inside the alpha support (the sorted tile lists)
  HDR_COSTS = 14,      // u32: a fused step has recorded every tile's duration (sticky)
  HDR_WORDS = 64
};
// Header magic: a workspace whose words 8-9 do not hold it has never been
// used (its sticky words may hold any leftover bytes) and is cleared.
constexpr uint32_t HDR_MAGIC0 = 0x67737248u, HDR_MAGIC1 = 0x2311B700u;

// Device pointers into the caller's workspace (computed on the host).
// ------------------------------------------------------- alpha support
//
// Tiles of a Gaussian's rectangle that it can reach with alpha >= alpha_min.
// Its alpha at a pixel is o exp(-Q/2), Q the conic quadratic form of the
// offset, so it reaches alpha_min only where Q <= t = 2 ln(o / alpha_min);
// a margin of 1e-4 on t keeps tiles where a float32 alpha could round up to
// alpha_min.  Inside one row of tiles the ellipse {Q <= t} meets a
// contiguous run of tiles: the x-range of the ellipse within the row's band
// of pixel-centre rows [16 ty, 16 ty + 15], mapped to the columns whose
// pixel centres [16 tx, 16 tx + 15] it overlaps.  Every input is a stored
// float32 value (centre as hi + lo, conic, opacity), so the projection
// kernel (parameters) and the emission kernel (per-pair test) agree with an
// FP64 reference evaluated in the same order.
struct Support {
  double U, V, t, hy, dys, ra;  // centre, level, half-height, dy of the rightmost point, 1 / a
};

__device__ inline bool support_of(float4 A, float4 B, float alpha_min, Support &s) {
#pragma clang fp contract(off)
  s.U = (double)A.x + (double)A.y;
  s.V = (double)A.z + (double)A.w;
  const double a = (double)B.x, b = (double)B.y, c = (double)B.z;
  const double det = a * c - b * b;
  s.t = 2.0 * log((double)B.w / (double)alpha_min) + 1e-4;
  if (!(det > 0.0) || !(s.t > 0.0)) return false;
  const double SA = c / det, SB = -b / det, SC = a / det;  // covariance
  s.hy = sqrt(s.t * SC);
  s.dys = SB * sqrt(s.t / SA);
  s.ra = 1.0 / a;
  return true;
}

// Run of tile columns of row ty (within [tx0, tx1]) reached by the support
// of the Gaussian with conic (a, b, c): returns its length and writes its
// first column to lo.
__device__ inline int support_row(const Support &s, double a, double b, double c, int ty, int tx0, int tx1,
                                  int &lo) {
#pragma clang fp contract(off)
  const double p = (double)(16 * ty) - s.V, q = (double)(16 * ty + 15) - s.V;
  if (q < -s.hy || p > s.hy) return 0;
  const double dr = fmin(fmax(s.dys, p), q), dl = fmin(fmax(-s.dys, p), q);
  const double br = b * dr, bl = b * dl;
  const double er = fmax(br * br - a * ((c * dr) * dr - s.t), 0.0);
  const double el = fmax(bl * bl - a * ((c * dl) * dl - s.t), 0.0);
  const double R = (-br + sqrt(er)) * s.ra, L = (-bl - sqrt(el)) * s.ra;
  const double clo = fmax(ceil(((s.U + L) - 15.0) * 0.0625), (double)tx0);
  const double chi = fmin(floor((s.U + R) * 0.0625), (double)tx1);
  if (!(clo <= chi)) return 0;
  lo = (int)clo;
  return (int)(chi - clo) + 1;
}

struct Workspace {
  uint32_t *hdr;
  float4 *recA;            // [n_rec] (u_hi, u_lo, v_hi, v_lo)
  float4 *recB;            // [n_rec] (conic a, b, c, opacity)
  float4 *recC;            // [n_rec] (r, g, b, camera-frame depth)
  uint4 *tinfo;            // [n_rec] (view tile offset, view TX | cull << 31, tx0 | tx1 << 16, ty0 | ty1 << 16)
  Support *support;        // [n_rec] alpha-support parameters (records with the cull bit)
  uint32_t *count;         // [n_rec] tiles touched (0 = culled)
  uint32_t *tile_visible;  // [depth-sort tiles] visible records of each projection block
  uint32_t *dkeys[2];      // [n_rec] depth keys (float32 bits), ping-pong
  uint32_t *dvals[2];      // [n_rec] record ids, ping-pong
  uint32_t *pkeys[2];      // [capacity] global tile ids, ping-pong
  uint32_t *pvals[2];      // [capacity] record ids, ping-pong
  uint32_t *hist;          // [RADIX][max_sort_tiles] digit counts per sort tile
  uint32_t *hoff;          // [RADIX][max_sort_tiles] exclusive scan of hist (digit-major)
  uint32_t *bucket_rec;    // [capacity / EMIT_BUCKET + 2] depth-order record holding pair EMIT_BUCKET * b
  uint32_t *digit_total;   // [RADIX]
  unsigned long long *whist;   // [RADIX][depth_tiles] pair counts per digit and tile (depth sort's last pass)
  unsigned long long *whoff;   // [RADIX][depth_tiles] exclusive scan of whist over the tiles
  unsigned long long *wdigit;  // [RADIX] pair counts per digit
  int2 *ranges;            // [total_tiles]
  float *T_final;          // [total_pixels]
  int32_t *last;           // [total_pixels]
  float *zr;               // [total_pixels] depth of the last blended entry (forward -> backward)
  unsigned long long *counts;  // [4] work totals (gsr_work_counts)
  double *grad2d;          // [n_rec][NGRAD2D], FP64 sums over tiles
  double *pose_part;       // [n_pose_blocks][n_views][6]
  uint32_t *queue;         // [total_tiles] work order of the persistent rasteriser
  unsigned long long *expand_bits;  // [chunks][8][4] adding step: one bit per pixel (ballot words)
  uint32_t *expand_cnt;    // [chunks] adding step: unreliable pixels per chunk, then their exclusive scan
  uint32_t *tile_cost;     // [total_tiles] duration of each tile in the last fused step (10 ns ticks)
  float *loss_part;        // [1] (unused slot kept for alignment)
  int dsorted;             // which depth buffer holds the sorted result
  int psorted;             // which pair buffer holds the sorted result
  // Packed pairs (when tile and record bits fit 32): one word per pair,
  // tile << pack_shift | record id, sorted without a value array; else
  // pack_shift = 0, keys hold tiles and pvals the record ids.
  int pack_shift;
  uint32_t id_mask;        // record id of a sorted word: word & id_mask
};

struct Plan {
  int64_t n = 0;
  int n_views = 0;
  int64_t n_rec = 0;
  int total_tiles = 0;
  int64_t total_pixels = 0;
  int64_t capacity = 0;
  int tile_bits = 0;
  int pack_shift = 0;      // record-id bits below the tile in a packed pair word (0: unpacked)
  int max_sort_tiles = 0;
  int depth_tiles = 0;     // sort tiles of the depth sort
  int n_pose_blocks = 0;
  size_t bytes = 0;
  // byte offsets inside the workspace
  size_t off_hdr, off_recA, off_recB, off_recC, off_rect, off_count, off_dkeys[2], off_dvals[2],
      off_pkeys[2], off_pvals[2], off_hist, off_digit, off_ranges, off_T, off_last, off_zr,
      off_grad2d, off_pose, off_queue, off_loss, off_counts, off_hoff, off_bucket, off_whist, off_whoff, off_wdigit,
      off_support, off_tile_visible, off_tile_cost, off_expand_bits, off_expand_cnt;
};

struct Tuning {
  int blocks_per_cu = 4;  // four blocks fit a CU (LDS): every resident slot busy
  int tiles_per_pop = 1;
  int lpt_order = 1;
  int batch = 192;  // records staged per forward round of the fused rasteriser (64, 128, 192, 256)
};

// Scalar renderer constants passed by value to kernels.
struct RenderConsts {
  float alpha_min, alpha_max, T_min;
  float bg[3];
  uint32_t grad_fields;  // bit f set: the backward accumulates grad2d field f
  uint32_t id_mask;      // record id of a sorted pair word (set by the launchers)
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ float wave_sum(float v) {
  // Butterfly over the 64 lanes of a wavefront.
  v += __shfl_xor(v, 32);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}

// Per-call header reset (one thread).  The overflow flag and required count
// are sticky until gsr_check_overflow reads them; on a workspace's first use
// (no magic yet) they are cleared too.
__device__ __forceinline__ void reset_header_words(uint32_t *hdr) {
  if (hdr[HDR_MAGIC] != HDR_MAGIC0 || hdr[HDR_MAGIC + 1] != HDR_MAGIC1) {
    hdr[HDR_REQUIRED] = 0u;
    hdr[HDR_REQUIRED + 1] = 0u;
    hdr[HDR_OVERFLOW] = 0u;
    hdr[HDR_COSTS] = 0u;
    hdr[HDR_MAGIC] = HDR_MAGIC0;
    hdr[HDR_MAGIC + 1] = HDR_MAGIC1;
  }
  hdr[HDR_NPAIRS] = 0u;
  hdr[HDR_NPAIRS + 1] = 0u;
  hdr[HDR_NVISIBLE] = 0u;
  hdr[HDR_NVISIBLE + 1] = 0u;
  hdr[HDR_NLISTED] = 0u;
  hdr[HDR_NLISTED + 1] = 0u;
  hdr[HDR_QUEUE] = 0u;
  hdr[HDR_FWD_DONE] = 1u;
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wavefront whose digit equals this lane's digit (and valid).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int nbits, uint64_t valid) {
  uint64_t m = valid;
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// --------------------------------------------------------------- tile order

// Log-scale bucket of a tile length (eight buckets per octave), 0 .. 255.
__device__ __forceinline__ uint32_t length_bucket(uint32_t x) {
  if (x == 0u) return 0u;
  const int b = 31 - __clz(x);  // floor(log2 x)
  const uint32_t m = b >= 3 ? (x >> (b - 3)) & 7u : (x << (3 - b)) & 7u;
  const uint32_t k = 1u + 8u * (uint32_t)b + m;
  return k < (uint32_t)RADIX ? k : (uint32_t)(RADIX - 1);
}

// Work order of the persistent rasteriser, computed by one block of NT
// threads: with `timed` (the last fused step on this workspace recorded every
// tile's duration in tile_cost) the tiles longest first, by a counting sort
// over length_bucket (order inside a bucket arbitrary; equal buckets inside a
// wavefront grouped by ballot matching, one LDS atomic per group); otherwise
// index order.  The queue is a permutation of the tiles whatever the recorded
// values.  `timed` must be the same in every thread; s_cnt, s_cur hold RADIX
// words and s_w NT / 64.
template <int NT>
__device__ __forceinline__ void order_tiles(const uint32_t *__restrict__ tile_cost, bool timed, int total,
                                            uint32_t *__restrict__ queue, uint32_t *s_cnt, uint32_t *s_cur,
                                            uint32_t *s_w) {
  static_assert(NT >= RADIX && NT % 64 == 0, "one thread per bucket, whole wavefronts");
  if (!timed) {
    for (int t = threadIdx.x; t < total; t += NT) queue[t] = (uint32_t)t;
    return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < RADIX) s_cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (int base = 0; base < total; base += NT) {
    const int t = base + (int)threadIdx.x;
    const bool valid = t < total;
    const uint32_t d = valid ? length_bucket(tile_cost[t]) : 0u;
    const uint64_t peers = match_digit(d, RADIX_BITS, __ballot(valid));
    if (valid && (peers & lanemask_lt()) == 0ull) atomicAdd(&s_cnt[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  // Start of each bucket: the tiles of all longer buckets (bucket RADIX - 1 - k
  // is the k-th in the order).
  {
    const int k = threadIdx.x;
    const uint32_t v = k < RADIX ? s_cnt[RADIX - 1 - k] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t pre = 0u;
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    if (k < RADIX) s_cur[RADIX - 1 - k] = pre + x - v;
  }
  __syncthreads();
  for (int base = 0; base < total; base += NT) {
    const int t = base + (int)threadIdx.x;
    const bool valid = t < total;
    const uint32_t d = valid ? length_bucket(tile_cost[t]) : 0u;
    const uint64_t peers = match_digit(d, RADIX_BITS, __ballot(valid));
    const int leader = __ffsll((long long)peers) - 1;
    uint32_t first = 0u;
    if (valid && lane == leader) first = atomicAdd(&s_cur[d], (uint32_t)__popcll(peers));
    first = __shfl(first, leader < 0 ? 0 : leader);
    if (valid) queue[first + (uint32_t)__popcll(peers & lanemask_lt())] = (uint32_t)t;
  }
}

// --------------------------------------------------------------- launchers (host)

// Preprocess (projection, binning data, depth keys) for every (view, Gaussian).
// Also resets the per-call header words, clears grad2d when clear_grad2d,
// zeroes *loss_zero when it is not null (start of a fused step), and writes
// the depth sort's first-pass digit counts into hist.
// With order_total > 0 it also writes the rasteriser's longest-first work
// order of that many tiles (from the durations the last fused step recorded).
void launch_preprocess(const gsr_gaussians &g, const gsr_camera *cams, const ViewInfo *views,
                       int n_views, const gsr_config &cfg, const Workspace &ws, bool clear_grad2d,
                       float *loss_zero, int max_sort_tiles, int order_total, hipStream_t s);

// Reliable-Gaussian selection (fine tracking stage).
void launch_select_reliable(const gsr_gaussians &g, const gsr_camera *cam, const float *depth, int W, int H,
                            float eps, float z_near, uint8_t *out, hipStream_t s);

// Sorting and list construction.
int launch_depth_sort(const Plan &p, Workspace &ws, hipStream_t s, int sort_grid);
void launch_emit_pairs(const Plan &p, const Workspace &ws, const ViewInfo *views, hipStream_t s);
int launch_pair_sort(const Plan &p, Workspace &ws, hipStream_t s, int sort_grid);
void launch_tile_ranges(const Plan &p, const Workspace &ws, hipStream_t s);
// Packed pairs: record ids of the sorted words into pvals[psorted].
void launch_unpack_ids(const Plan &p, const Workspace &ws, hipStream_t s);
void launch_fill_u32(uint32_t *ptr, uint32_t value, int64_t count, hipStream_t s);
void launch_fill_f32(float *ptr, float value, int64_t count, hipStream_t s);
void launch_reset_header(const Workspace &ws, hipStream_t s);
// The rasteriser's work order (order_tiles) as a one-block kernel.
void launch_queue_order(const Workspace &ws, int total_tiles, hipStream_t s);

// Rasterisation.
void launch_render_forward(const Plan &p, const Workspace &ws, const ViewInfo *views,
                           const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                           const gsr_images *out, hipStream_t s);
void launch_render_backward(const Plan &p, const Workspace &ws, const ViewInfo *views,
                            const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                            const float *g_rgb, const float *g_depth, const float *g_T,
                            hipStream_t s);
void launch_render_fused(const Plan &p, const Workspace &ws, const ViewInfo *views,
                         const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                         const float *t_rgb, const float *t_depth, const uint8_t *pmask,
                         float w_rgb, float w_depth, const float *loss_cap, const gsr_images *out, float *loss,
                         const Tuning &tun, int num_cus, hipStream_t s);
// Work totals of the last forward (re-walks its lists; needs the Gaussians'
// colours and the constants of that call).
void launch_work_counts(const Plan &p, const Workspace &ws, const ViewInfo *views, const int32_t *tile_view,
                        const gsr_gaussians &g, const RenderConsts &rc, hipStream_t s);
void launch_l1(const Plan &p, const ViewInfo *views, const float *rgb, const float *depth,
               const float *t_rgb, const float *t_depth, const uint8_t *pmask, float w_rgb,
               float w_depth, const float *loss_cap, float *g_rgb, float *g_depth, float *loss, hipStream_t s);
// Loss cap: factor x lower median of each view's per-pixel loss.
void launch_loss_median(const Plan &p, const ViewInfo *views, const float *px_loss, const uint8_t *pmask,
                        float factor, float *cap_out, hipStream_t s);

// Pose parameterisations (one thread per view).
void launch_pose_apply(int n, const float *xi, const gsr_camera *cin, gsr_camera *cout, hipStream_t s);
void launch_pose_xi_grad(int n, const float *xi, const float *d_pose, float *d_xi, hipStream_t s);
void launch_pose_from_qt(int n, const float *q, const float *t, const gsr_camera *cin, gsr_camera *cout,
                         hipStream_t s);
void launch_pose_qt_grad(int n, const float *q, const float *t, const float *d_pose, float *d_q, float *d_t,
                         hipStream_t s);

// Adaptive expansion (adding step over the planned views; deleting step).
void launch_expand_add(const Plan &p, const ViewInfo *views, const gsr_camera *cams, const float *T_final,
                       const float *depth, const float *depth_obs, const float *rgb_obs, float tau_T, float tau_D,
                       float scale_factor, float logit_init, const Workspace &ws, int64_t n, int64_t capacity,
                       const gsr_gaussians_out &out, uint8_t *pixel_flag, int64_t *count, hipStream_t s);
void launch_expand_delete(const gsr_gaussians &g, const gsr_camera *cam, const float *depth_obs, int W, int H,
                          float gamma, float eta, float z_near, float *logit_out, uint8_t *decayed, hipStream_t s);

// Backward preprocess (chain to parameters and pose).
void launch_preprocess_backward(const Plan &p, const gsr_gaussians &g, const gsr_camera *cams,
                                const gsr_config &cfg, const Workspace &ws, const gsr_grads &gr,
                                hipStream_t s);

}  // namespace gsr
