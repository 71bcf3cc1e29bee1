// Per-tile compositing: front-to-back alpha blending of colour and depth
// (GS-SLAM Eq. 4-5), its backward pass (supplement eq. grad_depth and the
// colour analogue), and the weighted L1 loss gradient (Eq. 6 / Eq. 10).
//
// One 256-thread block (four wave64) renders one 16x16 tile, one thread per
// pixel.  The tile's Gaussians are staged through LDS in batches: each
// thread loads one record, converts its centre to tile-relative FP32
// coordinates (the record keeps the centre as a float pair, so the offset to
// a pixel keeps full precision even at x ~ 1000 px), and pre-scales the
// conic so that alpha = min(alpha_max, o * 2^P) with
// P = a'' dx^2 + 2 b'' dx dy + c'' dy^2 and (a'', b'', c'') = -log2(e)/2 * conic
// (the staged record holds 2 b'').  The forward and the backward evaluate
// alpha with the same inlined function and contraction disabled, so both
// take every threshold decision identically.
#pragma clang fp contract(off)

#include "gsr_internal.h"

namespace gsr {

constexpr int BATCH = 192;  // staged records per forward round (<= BLOCK; the fused kernel's is tunable)
constexpr float NEG_HALF_LOG2E = -0.72134752044448170368f;  // -log2(e) / 2
constexpr float LN2 = 0.69314718055994530942f;
// Alpha threshold of a pixel that has stopped (or lies outside the image):
// above any alpha (alpha <= alpha_max <= 1) and an inline constant of the
// instruction set, so that no register holds it.
constexpr float A_STOPPED = 2.f;

struct Staged {
  float4 geo;  // (u_rel, v_rel, opacity, depth)
  float4 con;  // (a'', 2 b'', c'', unused)
  float4 col;  // (r, g, b, unused)
};

struct TileInfo {
  int view;
  int tx, ty;
  int W, H;
  int64_t pix;     // global pixel index of this thread (valid if inside)
  int64_t HW;      // pixels of the view
  int64_t pix_off; // first pixel of the view
  bool inside;
  int2 range;
  float x0, y0;
};

__device__ __forceinline__ TileInfo tile_info(int tile, const ViewInfo *__restrict__ views,
                                              const int32_t *__restrict__ tile_view,
                                              const int2 *__restrict__ ranges) {
  TileInfo ti;
  ti.view = tile_view[tile];
  const ViewInfo vi = views[ti.view];
  const int local = tile - vi.tile_off;
  ti.ty = local / vi.TX;
  ti.tx = local - ti.ty * vi.TX;
  ti.W = vi.W;
  ti.H = vi.H;
  const int px = ti.tx * TILE + (threadIdx.x & (TILE - 1));
  const int py = ti.ty * TILE + (threadIdx.x >> 4);
  ti.inside = px < vi.W && py < vi.H;
  ti.HW = (int64_t)vi.W * vi.H;
  ti.pix_off = vi.pix_off;
  ti.pix = vi.pix_off + (int64_t)py * vi.W + px;
  ti.range = ranges[tile];
  ti.x0 = (float)(ti.tx * TILE);
  ti.y0 = (float)(ti.ty * TILE);
  return ti;
}

// Load record `id` into this thread's staging slot (three 16-byte loads).
__device__ __forceinline__ Staged stage_record(uint32_t id, float x0, float y0, const float4 *__restrict__ recA,
                                               const float4 *__restrict__ recB,
                                               const float4 *__restrict__ recC) {
  const float4 A = recA[id];
  const float4 Bc = recB[id];
  const float4 C = recC[id];
  Staged s;
  // (u_hi - x0) is exact for |u_hi| < 2^24 and integer x0; the low word adds
  // the remaining bits.
  s.geo = make_float4((A.x - x0) + A.y, (A.z - y0) + A.w, Bc.w, C.w);
  s.con = make_float4(NEG_HALF_LOG2E * Bc.x, 2.f * (NEG_HALF_LOG2E * Bc.y), NEG_HALF_LOG2E * Bc.z, 0.f);
  s.col = make_float4(C.x, C.y, C.z, 0.f);
  return s;
}

// alpha of a staged Gaussian at pixel offset (dx, dy) = centre - pixel;
// oG >= 0, so the clamp to [0, alpha_max] is min(oG, alpha_max).
__device__ __forceinline__ float splat_alpha(const float4 &geo, const float4 &con, float dx, float dy,
                                             float alpha_max, float &G, float &oG) {
  const float t = __fmaf_rn(con.x, dx, con.y * dy);
  const float P = __fmaf_rn(con.z * dy, dy, dx * t);
  G = __builtin_amdgcn_exp2f(P);
  oG = geo.z * G;
  return __builtin_amdgcn_fmed3f(oG, 0.f, alpha_max);
}

// ------------------------------------------------------------------ forward

struct FwdState {
  float T, C0, C1, C2, D;
  int last;
  float zr;  // depth of the last blended entry (0 if none): the backward's reference depth
};

// Depth of list entry pos of the tile, from the staged batch that starts at
// entry lo when it holds pos, else from the record.
__device__ __forceinline__ float entry_depth(int pos, int lo, const Staged *s_rec, const TileInfo &ti,
                                            const uint32_t *__restrict__ ids, const float4 *__restrict__ recC,
                                            uint32_t id_mask) {
  if (pos >= lo) return s_rec[pos - lo].geo.w;
  return recC[ids[ti.range.x + pos] & id_mask].w;
}

// With COUNT, the walk also adds its work to counts (wave totals, once per
// tile): counts[1] += list entries examined by live pixels (including the
// entry that stopped a pixel), counts[2] += entries blended.  The render
// kernels do not count; gsr_work_counts re-walks the lists with counting on.
template <bool COUNT, int NB = BATCH>
__device__ __forceinline__ void tile_forward(const TileInfo &ti, int64_t n, const float4 *__restrict__ recA,
                                             const float4 *__restrict__ recB,
                                             const float4 *__restrict__ recC,
                                             const uint32_t *__restrict__ ids, const RenderConsts &rc,
                                             Staged *s_rec, FwdState &st, unsigned long long *counts,
                                             uint32_t *s_id = nullptr, int *staged_lo = nullptr) {
  st.T = 1.f;
  st.C0 = st.C1 = st.C2 = st.D = 0.f;
  st.last = 0;
  st.zr = 0.f;
  // The pixel's alpha threshold; A_STOPPED once it has stopped (or outside
  // the image), so that no later entry is accepted.
  float amin = ti.inside ? rc.alpha_min : A_STOPPED;
  int lo_last = -1;  // first entry of the staged batch (-1: none staged)
  uint32_t nev_w = 0u, nbl_w = 0u;
  const float lx = (float)(threadIdx.x & (TILE - 1));
  const float ly = (float)(threadIdx.x >> 4);
  // This thread's list word of the next batch, loaded one batch ahead.
  uint32_t next_id = 0u;
  static_assert(NB % 64 == 0 && NB <= BLOCK, "whole wavefronts of staging threads");
  if ((int)threadIdx.x < NB && ti.range.x + (int)threadIdx.x < ti.range.y) next_id = ids[ti.range.x + threadIdx.x];
  for (int base = ti.range.x; base < ti.range.y; base += NB) {
    if (__syncthreads_and(amin == A_STOPPED)) break;
    const int pos = base + threadIdx.x;
    if ((int)threadIdx.x < NB && pos < ti.range.y) {
      const uint32_t id = next_id & rc.id_mask;
      if (s_id) s_id[threadIdx.x] = id;
      s_rec[threadIdx.x] = stage_record(id, ti.x0, ti.y0, recA, recB, recC);
      if (pos + NB < ti.range.y) next_id = ids[pos + NB];
    }
    lo_last = base - ti.range.x;
    __syncthreads();
    // Branch-free walk: every lane evaluates every entry and keeps or drops
    // the result with selects; the wave leaves the batch once all of its
    // pixels have stopped.  `live` (wave-uniform) holds the lanes still
    // blending.
    const int cnt = min(NB, ti.range.y - base);
    uint64_t live = __builtin_amdgcn_ballot_w64(amin != A_STOPPED);
    for (int k = 0; k < cnt && live; ++k) {
      if (COUNT) nev_w += (uint32_t)__popcll(live);
      const float4 geo = s_rec[k].geo;
      const float4 con = s_rec[k].con;
      const float dx = geo.x - lx, dy = geo.y - ly;
      float G, oG;
      const float alpha = splat_alpha(geo, con, dx, dy, rc.alpha_max, G, oG);
      const bool acc = alpha >= amin;
      // Blend weight alpha T and the transmittance behind, T - alpha T.
      const float wa = alpha * st.T;
      const float Tn = st.T - wa;
      const bool stop = acc && Tn < rc.T_min;
      const bool blend = acc && !stop;
      if (COUNT) nbl_w += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(blend));
      amin = stop ? A_STOPPED : amin;
      // Nearly every entry blends in some lane: no branch around the update.
      const float4 col = s_rec[k].col;
      const float w = blend ? wa : 0.f;
      st.C0 = __fmaf_rn(w, col.x, st.C0);
      st.C1 = __fmaf_rn(w, col.y, st.C1);
      st.C2 = __fmaf_rn(w, col.z, st.C2);
      st.D = __fmaf_rn(w, geo.w, st.D);
      st.T = blend ? Tn : st.T;
      st.last = blend ? base - ti.range.x + k + 1 : st.last;
      live = __builtin_amdgcn_ballot_w64(amin != A_STOPPED);
    }
  }
  if (staged_lo) *staged_lo = lo_last;
  // The reference depth: the last blended entry's, read once per pixel (an
  // entry was blended, so a batch was staged).
  if (st.last > 0) st.zr = entry_depth(st.last - 1, lo_last, s_rec, ti, ids, recC, rc.id_mask);
  if (COUNT && __lane_id() == 0 && nev_w) {
    atomicAdd(counts + 1, (unsigned long long)nev_w);
    atomicAdd(counts + 2, (unsigned long long)nbl_w);
  }
  st.C0 = __fmaf_rn(st.T, rc.bg[0], st.C0);
  st.C1 = __fmaf_rn(st.T, rc.bg[1], st.C1);
  st.C2 = __fmaf_rn(st.T, rc.bg[2], st.C2);
}

// ----------------------------------------------------------------- backward
//
// Per list entry the backward needs, summed over the 256 pixels of the tile,
//   S1 = sum dLdP, Sx = sum dLdP dx, Sy = sum dLdP dy,
//   Sxx = sum dLdP dx^2, Sxy = sum dLdP dx dy, Syy = sum dLdP dy^2,
//   Sc = sum w gC_c (c = r, g, b), Sd = sum w gD,
// with dx = u - x, dy = v - y.  Expanding dx, dy about the tile centre turns
// all of them into moments of two per-pixel values (dLdP and w) against
// per-pixel constants: the matrix [dLdP; w] (entries x pixels) times the
// matrix [1, xc, yc, xc^2, xc yc, yc^2, gC_r, gC_g, gC_b, gD] (pixels x 10),
// a dense contraction over the pixels.  Each wavefront collects dLdP and w of
// 8 entries (16 rows) for its 64 pixels in LDS and contracts them on the
// bf16 matrix cores (v_mfma_f32_16x16x32_bf16, each value split into two
// bf16 halves: K = 128 slots in 4 steps); the four
// wavefronts add their 16x16 products into the block's per-entry sums.

constexpr int SUB = 64;                   // entries per backward sub-batch
constexpr int MA_ROWS = 16;               // 8 entries x (dLdP, w)
constexpr int MA_STRIDE = 64 + 4;         // 32-bit words (bf16 pairs) per row (padding spreads LDS banks)
constexpr int MA_WAVE = MA_ROWS * MA_STRIDE;
constexpr int NMOM = 10;                  // per-entry sums kept in LDS

typedef float float4v __attribute__((ext_vector_type(4)));

struct BwdIn {
  float T;         // final transmittance
  int last;        // list positions [0, last) to walk
  float zr;        // depth of the last contributor (0 if none)
  float gC0, gC1, gC2, gD, gT;
  // The fused step's upstream colour and depth gradients divided by their
  // weights (sC = gC / w_rgb, sD = gD / w_depth), values that bf16 holds
  // exactly (signs of the L1 residuals).
  float sC0, sC1, sC2, sD;
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Contract the wave's collected rows (rows 2q = dLdP, 2q+1 = w of entry q)
// with the per-pixel constants on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16): every per-pixel value x of the A rows is held
// as a pair (h, l) of bf16, h = x with the low 16 bits of its float32 cleared
// and l = x - h rounded to bf16 (h + l carries 16 significant bits, a
// relative error below 2^-16), and the pair occupies two consecutive K slots
// whose B entries both hold the pixel's column value (exact in bf16 for the
// moment polynomials of half-integer coordinates, at most 8 significant
// bits, and for residual signs).  K = 128 slots (64 pixels x 2) in 4 steps;
// step j covers the wave's pixel row j.  Lane l supplies A[l % 16][k] and
// B[k][l % 16] for the 8 slots k of its group l / 16; D[i][l % 16] lands in
// register i % 4 of lane 16 (i / 4) + l % 16.  The accumulation is FP32.
// The result is consumed (mfma_consume) only at the next group, so the
// matrix-core chain runs while the wavefront walks on.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t split_bf16(float x) {
  const float h = __uint_as_float(__float_as_uint(x) & 0xFFFF0000u);
  const float2v p = {h, x - h};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(p, bf16x2));
}

// With BLO the B values are not exact in bf16: Bl holds the low halves
// (B - Bb rounded to bf16) and a second set of steps adds A Bl, so that the
// products keep about 16 significant bits on both sides.
template <bool BLO>
__device__ __forceinline__ float4v mfma_issue_split(const float *mA, const bf16x8 Bb[4], const bf16x8 *Bl) {
  const int lane = __lane_id();
  const int r = lane & 15, g = lane >> 4;
  wave_lds_sync();
  // Lane (g, r): row r, words (pixels) 16 j + 4 g .. + 3 of step j.
  const uint4 *src = reinterpret_cast<const uint4 *>(mA + r * MA_STRIDE + 4 * g);
  const uint4 a0 = src[0], a1 = src[4], a2 = src[8], a3 = src[12];
  float4v D = {0.f, 0.f, 0.f, 0.f};
  D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a0), Bb[0], D, 0, 0, 0);
  D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a1), Bb[1], D, 0, 0, 0);
  D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a2), Bb[2], D, 0, 0, 0);
  D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a3), Bb[3], D, 0, 0, 0);
  if constexpr (BLO) {
    D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a0), Bl[0], D, 0, 0, 0);
    D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a1), Bl[1], D, 0, 0, 0);
    D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a2), Bl[2], D, 0, 0, 0);
    D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a3), Bl[3], D, 0, 0, 0);
  }
  return D;
}

// Store the useful products of a contraction of nq entries into the
// wavefront's own per-entry sums s_sum[entry][NMOM] (entry q's slot in byte
// q of slots; a wavefront meets each entry once per sub-batch, so plain
// stores suffice and the four wavefronts never contend for an address).
// Lane (g, col) holds rows 4g..4g+3: entry 2g (dLdP row, w row) and entry
// 2g+1.  Columns 0-5 are taken from the dLdP rows, 6-9 from the w rows.
__device__ __forceinline__ void mfma_consume(const float4v &D, int nq, uint64_t slots, float *s_sum) {
  const int lane = __lane_id();
  const int g = lane >> 4;
  const int col = lane & 15;
  if (col < NMOM) {
    const bool mom = col < 6;
    const int q0 = 2 * g, q1 = 2 * g + 1;
    if (q0 < nq) s_sum[(int)((slots >> (8 * q0)) & 255u) * NMOM + col] = mom ? D[0] : D[1];
    if (q1 < nq) s_sum[(int)((slots >> (8 * q1)) & 255u) * NMOM + col] = mom ? D[2] : D[3];
  }
}

// Walk the tile's list back to front; per entry, dLdP and w of every pixel
// go through the contraction above, and the flush turns the per-entry sums
// into the 2D gradients, added to grad2d with one FP64 atomic per field (a
// Gaussian that covers many tiles sums partials of both signs; the FP64 sum
// keeps the result independent of the order the tiles finish in).  grad2d
// fields: (u, v, conic a, b, c, opacity, r, g, b, depth).
//
// The per-entry sums run on the bf16 matrix cores (mfma_issue_split).
// Without BLO (the fused step) the upstream columns are the residual signs
// in.sC / in.sD and the colour and depth sums are scaled by w_rgb and
// w_depth at the flush; with BLO (the separate backward, any upstream
// gradient) they are in.gC / in.gD themselves, split into high and low bf16
// halves like the A values.
template <bool BLO>
__device__ __forceinline__ void tile_backward(const TileInfo &ti, int64_t n, const float4 *__restrict__ recA,
                                              const float4 *__restrict__ recB,
                                              const float4 *__restrict__ recC,
                                              const uint32_t *__restrict__ ids, const RenderConsts &rc,
                                              const BwdIn &in, double *__restrict__ grad2d,
                                              Staged *s_rec, float *s_part, uint32_t *s_id, int *s_max,
                                              float *s_mA, int staged_lo = -1, float w_rgb = 1.f,
                                              float w_depth = 1.f) {
  const float lx = (float)(threadIdx.x & (TILE - 1));
  const float ly = (float)(threadIdx.x >> 4);
  const int lane = __lane_id();
  const int wv = threadIdx.x >> 6;
  float *mA = s_mA + wv * MA_WAVE;
  float *my_part = s_part + wv * SUB * NMOM;  // this wavefront's per-entry sums
  if (threadIdx.x == 0) *s_max = 0;
  __syncthreads();
  if (in.last > 0) atomicMax(s_max, in.last);
  __syncthreads();
  const int maxlast = *s_max;
  if (maxlast == 0) return;

  // Per-pixel constants of the contraction, in the B-operand layout,
  // coordinates relative to the tile centre.  The upstream gradients reach
  // those lanes through the wave's LDS rows.
  bf16x8 Bb[4];
  bf16x8 Bl[BLO ? 4 : 1];
  {
    // Step j, lane (g, col): elements 2 i and 2 i + 1 hold column col of
    // pixel x = 4 g + i of the wave's row j (y = 4 wv + j).
    mA[0 * MA_STRIDE + lane] = BLO ? in.gC0 : in.sC0;
    mA[1 * MA_STRIDE + lane] = BLO ? in.gC1 : in.sC1;
    mA[2 * MA_STRIDE + lane] = BLO ? in.gC2 : in.sC2;
    mA[3 * MA_STRIDE + lane] = BLO ? in.gD : in.sD;
    wave_lds_sync();
    // Rebuilt per tile from an opaque copy of the lane index: kept out of
    // the tile loop, these tile-invariant values would be held in registers
    // (or spilled) across the forward walk.
    int lane_t = lane;
    __asm__ volatile("" : "+v"(lane_t));
    const int col = lane_t & 15, g = lane_t >> 4;
    const bool up = col >= 6 && col < NMOM;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float yc = (float)(4 * wv + j) - 7.5f;
      const float4 q = *reinterpret_cast<const float4 *>(mA + (up ? col - 6 : 0) * MA_STRIDE + 16 * j + 4 * g);
      const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float xc = (float)(4 * g + i) - 7.5f;
        // Columns 1, xc, yc, xc^2, xc yc, yc^2, then the upstream values.
        const float a = col == 1 || col == 3 || col == 4 ? xc : (col == 2 || col == 5 ? yc : 1.f);
        const float b = col == 3 ? xc : (col == 4 || col == 5 ? yc : 1.f);
        const float x = up ? qv[i] : (col < 6 ? a * b : 0.f);
        const __bf16 v = (__bf16)x;
        Bb[j][2 * i] = v;
        Bb[j][2 * i + 1] = v;
        if constexpr (BLO) {
          const __bf16 vl = (__bf16)(x - (float)v);
          Bl[j][2 * i] = vl;
          Bl[j][2 * i + 1] = vl;
        }
      }
    }
    wave_lds_sync();
  }

  float T = in.T;
  const float Tf = in.T;
  // Blend behind the current entry, normalised by the transmittance in front
  // of it, enters dL/dalpha only through the upstream-weighted scalar
  //   S = gC . aC + gD . aDs,
  // (aC: colour behind, starting at the background; aDs: depth behind,
  // relative to the depth zr of the pixel's last contributor), which obeys
  // the same recurrence S <- S + alpha (Q - S) with Q = gC . c + gD (z - zr).
  // With the telescoping identity sum_m alpha_m T_m = 1 - T_f,
  //   dL/dalpha_k = T_k (Q_k - S_k) + (gD zr - gT) T_f / (1 - alpha_k).
  // On a surface all depths agree to a few mm, so the shifted terms keep
  // their float32 digits (z_k - aD_k itself would cancel).
  float S = in.gC0 * rc.bg[0] + in.gC1 * rc.bg[1] + in.gC2 * rc.bg[2];
  const float zr = in.zr;
  const float Kf = (in.gD * zr - in.gT) * Tf;

  // Sub-batches [b SUB, (b + 1) SUB), walked from the last one that holds
  // an entry below maxlast.  Those inside the forward's last batch (still
  // staged, records and ids, from list position staged_lo on) are read in
  // place; the others are staged into the first SUB slots.
  uint32_t next_id = 0u;  // list word of this thread's slot in sub-batch next_lo, loaded ahead
  int next_lo = -1;
  for (int lo = ((maxlast - 1) / SUB) * SUB; lo >= 0; lo -= SUB) {
    const int hi = min(lo + SUB, maxlast);
    const int cnt = hi - lo;
    int off = 0;  // slot of entry lo in s_rec / s_id
    if (staged_lo >= 0 && lo >= staged_lo) {
      off = lo - staged_lo;
    } else {
      staged_lo = -1;
      if ((int)threadIdx.x < cnt) {
        const uint32_t id = (next_lo == lo ? next_id : ids[ti.range.x + lo + threadIdx.x]) & rc.id_mask;
        s_id[threadIdx.x] = id;
        s_rec[threadIdx.x] = stage_record(id, ti.x0, ti.y0, recA, recB, recC);
      }
    }
    if (lo >= SUB && !(staged_lo >= 0 && lo - SUB >= staged_lo)) {
      if ((int)threadIdx.x < SUB) next_id = ids[ti.range.x + lo - SUB + threadIdx.x];
      next_lo = lo - SUB;
    }
    {
      // Entries without a contribution in this wavefront keep zero sums.
      float4 *z = reinterpret_cast<float4 *>(my_part);
      for (int k = lane; k < SUB * NMOM / 4; k += 64) z[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    int nq = 0;
    uint64_t slots = 0;
    float4v pD = {0.f, 0.f, 0.f, 0.f};  // contraction of the previous group, not yet added
    int p_nq = 0;
    uint64_t p_slots = 0;
    // One step past the batch (k = lo - 1) contracts the last partial group.
    for (int k = hi - 1; k >= lo - 1; --k) {
      const int j = k - lo;
      if (k >= lo) {
        const float4 geo = s_rec[off + j].geo;
        const float4 con = s_rec[off + j].con;
        const float dx = geo.x - lx, dy = geo.y - ly;
        float G, oG;
        const float alpha = splat_alpha(geo, con, dx, dy, rc.alpha_max, G, oG);
        const bool has = k < in.last && alpha >= rc.alpha_min;
        // Wave-uniform guard; inside it every lane computes and the lanes
        // without a contribution are masked with selects (NaN-safe).
        if (__any(has)) {
          const float4 col = s_rec[off + j].col;
          // Lanes without a contribution take alpha = 0, which leaves T and
          // S unchanged (1 / (1 - 0) is exactly 1) and gives w = 0.
          const float ae = has ? alpha : 0.f;
          const float rinv = __builtin_amdgcn_rcpf(1.f - ae);
          const float Tk = T * rinv;  // transmittance in front of this Gaussian
          T = Tk;
          const float w = ae * Tk;
          const float Q = __fmaf_rn(in.gD, geo.w - zr, __fmaf_rn(in.gC2, col.z, __fmaf_rn(in.gC1, col.y, in.gC0 * col.x)));
          const float QS = Q - S;
          const float dLda = __fmaf_rn(Tk, QS, Kf * rinv);
          S = __fmaf_rn(ae, QS, S);
          const bool open = has && oG <= rc.alpha_max;
          // dL/dP with G = 2^P (the ln 2 and the conic pre-scale are applied
          // at the flush); dL/d(opacity) = dLdP / o there.
          const float dLdP = open ? dLda * oG : 0.f;
          uint32_t *mw = reinterpret_cast<uint32_t *>(mA);
          mw[(2 * nq) * MA_STRIDE + lane] = split_bf16(dLdP);
          mw[(2 * nq + 1) * MA_STRIDE + lane] = split_bf16(w);
          slots |= (uint64_t)j << (8 * nq);
          ++nq;
        }
      }
      if (nq == 8 || (k < lo && nq > 0)) {
        if (p_nq > 0) mfma_consume(pD, p_nq, p_slots, my_part);
        pD = mfma_issue_split<BLO>(mA, Bb, Bl);
        p_nq = nq;
        p_slots = slots;
        nq = 0;
        slots = 0;
        // The rows were read into registers; the next group may rewrite them.
        wave_lds_sync();
      }
    }
    if (p_nq > 0) mfma_consume(pD, p_nq, p_slots, my_part);
    __syncthreads();
    // Flush.  First one thread per Gaussian of the batch converts its sums:
    // with the centre relative to the tile centre (uc, vc) and the pixel
    // moments M about it,
    //   Sx = uc M1 - Mx, Sy = vc M1 - My, Sxx = uc^2 M1 - 2 uc Mx + Mxx,
    //   Sxy = uc vc M1 - uc My - vc Mx + Mxy, Syy = vc^2 M1 - 2 vc My + Myy;
    // then dL/du = 2 ln2 (a'' Sx + b'' Sy), dL/dv = 2 ln2 (b'' Sx + c'' Sy)
    // with the pre-scaled conic (a'', b'', c'') = -log2(e)/2 (a, b, c), and
    //   dL/da = -Sxx/2, dL/db = -Sxy, dL/dc = -Syy/2, dL/do = M1 / o.
    // Then the block adds them to grad2d field-parallel: consecutive lanes
    // take consecutive fields of one Gaussian, so each atomic instruction
    // touches a few contiguous 80-byte rows.
    double *s_out = reinterpret_cast<double *>(s_mA);  // [SUB][NGRAD2D], free during the flush
    if ((int)threadIdx.x < cnt) {
      // The four wavefronts' sums, added in a fixed order.
      const float *src = s_part + threadIdx.x * NMOM;
      double m[NMOM];
#pragma unroll
      for (int f = 0; f < NMOM; ++f)
        m[f] = (double)((src[f] + src[SUB * NMOM + f]) + (src[2 * SUB * NMOM + f] + src[3 * SUB * NMOM + f]));
      const Staged &sr = s_rec[off + threadIdx.x];
      const double uc = (double)sr.geo.x - 7.5, vc = (double)sr.geo.y - 7.5;
      const double M1 = m[0], Mx = m[1], My = m[2], Mxx = m[3], Mxy = m[4], Myy = m[5];
      const double Sx = uc * M1 - Mx, Sy = vc * M1 - My;
      const double Sxx = (uc * uc * M1 - 2.0 * uc * Mx) + Mxx;
      const double Sxy = ((uc * vc * M1 - uc * My) - vc * Mx) + Mxy;
      const double Syy = (vc * vc * M1 - 2.0 * vc * My) + Myy;
      const double a2 = (double)sr.con.x, b2 = 0.5 * (double)sr.con.y, c2 = (double)sr.con.z;
      double *o = s_out + threadIdx.x * NGRAD2D;
      o[0] = 2.0 * (double)LN2 * (a2 * Sx + b2 * Sy);
      o[1] = 2.0 * (double)LN2 * (b2 * Sx + c2 * Sy);
      o[2] = -0.5 * Sxx;
      o[3] = -Sxy;
      o[4] = -0.5 * Syy;
      o[5] = M1 / (double)sr.geo.z;
      constexpr bool SCALED = !BLO;  // the upstream columns were the residual signs
      o[6] = SCALED ? m[6] * (double)w_rgb : m[6];
      o[7] = SCALED ? m[7] * (double)w_rgb : m[7];
      o[8] = SCALED ? m[8] * (double)w_rgb : m[8];
      o[9] = SCALED ? m[9] * (double)w_depth : m[9];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt * NGRAD2D; t += BLOCK) {
      const int e = t / NGRAD2D, f = t - e * NGRAD2D;
      const double v = s_out[t];
      if (v != 0.0 && ((rc.grad_fields >> f) & 1u)) atomicAdd(grad2d + (size_t)s_id[off + e] * NGRAD2D + f, v);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ kernels

struct RasterArgs {
  const float4 *recA;
  const float4 *recB;
  const float4 *recC;  // (r, g, b, camera-frame depth) per record
  const uint32_t *ids;
  const int2 *ranges;
  const ViewInfo *views;
  const int32_t *tile_view;
  int64_t n;
  RenderConsts rc;
};

// Raster arguments of a workspace: the sorted pair words and the mask that
// extracts a record id from them.
static RasterArgs raster_args(const Workspace &ws, const ViewInfo *views, const int32_t *tile_view,
                              const gsr_gaussians &g, RenderConsts rc) {
  rc.id_mask = ws.id_mask;
  const uint32_t *ids = ws.pack_shift ? ws.pkeys[ws.psorted] : ws.pvals[ws.psorted];
  return RasterArgs{ws.recA, ws.recB, ws.recC, ids, ws.ranges, views, tile_view, g.n, rc};
}

// Per-pixel forward state that a separate backward reads (the unfused
// forward); all null in the fused step, whose backward keeps it in registers.
struct PixelState {
  float *T;
  int32_t *last;
  float *zr;
};

__device__ __forceinline__ void save_state(const PixelState &ps, int64_t pix, const FwdState &st) {
  if (ps.T) ps.T[pix] = st.T;
  if (ps.last) ps.last[pix] = st.last;
  if (ps.zr) ps.zr[pix] = st.zr;
}

__global__ __launch_bounds__(BLOCK) void k_render_fwd(RasterArgs a, PixelState ps, gsr_images out) {
  __shared__ Staged s_rec[BATCH];
  const TileInfo ti = tile_info(blockIdx.x, a.views, a.tile_view, a.ranges);
  FwdState st;
  tile_forward<false>(ti, a.n, a.recA, a.recB, a.recC, a.ids, a.rc, s_rec, st, nullptr);
  if (!ti.inside) return;
  save_state(ps, ti.pix, st);
  const int64_t loc = ti.pix - ti.pix_off;
  if (out.rgb) {
    float *o = out.rgb + 3 * ti.pix_off + loc;
    o[0] = st.C0;
    o[ti.HW] = st.C1;
    o[2 * ti.HW] = st.C2;
  }
  if (out.depth) out.depth[ti.pix] = st.D;
  if (out.T_final) out.T_final[ti.pix] = st.T;
  if (out.last) out.last[ti.pix] = st.last;
}

__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_render_bwd(RasterArgs a, const float *__restrict__ T_ws,
                                                      const int32_t *__restrict__ last_ws,
                                                      const float *__restrict__ zr_ws,
                                                      const float *__restrict__ g_rgb,
                                                      const float *__restrict__ g_depth,
                                                      const float *__restrict__ g_T,
                                                      double *__restrict__ grad2d) {
  // Without a forward in the same kernel the walk stages SUB entries at a time.
  __shared__ Staged s_rec[SUB];
  __shared__ float s_part[4 * SUB * NMOM];
  __shared__ uint32_t s_id[SUB];
  __shared__ int s_max;
  __shared__ __align__(16) float s_mA[4 * MA_WAVE];
  const TileInfo ti = tile_info(blockIdx.x, a.views, a.tile_view, a.ranges);
  BwdIn in{1.f, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (ti.inside) {
    const int64_t loc = ti.pix - ti.pix_off;
    in.zr = zr_ws[ti.pix];
    in.T = T_ws[ti.pix];
    in.last = last_ws[ti.pix];
    const float *gc = g_rgb + 3 * ti.pix_off + loc;
    in.gC0 = gc[0];
    in.gC1 = gc[ti.HW];
    in.gC2 = gc[2 * ti.HW];
    in.gD = g_depth ? g_depth[ti.pix] : 0.f;
    in.gT = g_T ? g_T[ti.pix] : 0.f;
  }
  tile_backward<true>(ti, a.n, a.recA, a.recB, a.recC, a.ids, a.rc, in, grad2d, s_rec, s_part, s_id,
                            &s_max, s_mA);
}

__device__ __forceinline__ float sgnf(float x) { return (float)((x > 0.f) - (x < 0.f)); }

// Persistent fused step: blocks take tiles from an atomic counter (in index
// order, or in the longest-first order of `queue`); per tile run the
// forward blend, the L1 loss gradient of every pixel, and the backward walk
// without leaving the block (per-pixel state stays in registers).  Each
// tile's duration goes to tile_cost, the next step's longest-first order.
template <int NB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_render_fused(RasterArgs a, uint32_t *__restrict__ hdr,
                                                        const uint32_t *__restrict__ queue, int total_tiles,
                                                        int tiles_per_pop, const float *__restrict__ t_rgb,
                                                        const float *__restrict__ t_depth,
                                                        const uint8_t *__restrict__ pmask, float w_rgb,
                                                        float w_depth, const float *__restrict__ loss_cap,
                                                        gsr_images out, float *__restrict__ loss,
                                                        double *__restrict__ grad2d, PixelState ps,
                                                        uint32_t *__restrict__ tile_cost) {
  __shared__ Staged s_rec[NB];
  __shared__ float s_part[4 * SUB * NMOM];
  __shared__ uint32_t s_id[NB];
  __shared__ int s_max;
  __shared__ __align__(16) float s_mA[4 * MA_WAVE];
  __shared__ int s_q;
  __shared__ float s_loss[4];
  for (;;) {
    if (threadIdx.x == 0) s_q = (int)atomicAdd(hdr + HDR_QUEUE, (uint32_t)tiles_per_pop);
    __syncthreads();
    const int q0 = s_q;
    __syncthreads();
    if (q0 >= total_tiles) break;
    const int q1 = min(q0 + tiles_per_pop, total_tiles);
    for (int q = q0; q < q1; ++q) {
      const int tile = queue ? (int)queue[q] : q;
      const TileInfo ti = tile_info(tile, a.views, a.tile_view, a.ranges);
      const uint64_t clk0 = wall_clock64();
      // The pixel's targets, loaded before the forward walk hides their latency.
      float tc0 = 0.f, tc1 = 0.f, tc2 = 0.f, td = 0.f, cap = __builtin_inff();
      bool m = false;
      if (ti.inside) {
        const float *tc = t_rgb + 3 * ti.pix_off + (ti.pix - ti.pix_off);
        tc0 = tc[0];
        tc1 = tc[ti.HW];
        tc2 = tc[2 * ti.HW];
        td = t_depth[ti.pix];
        m = pmask ? pmask[ti.pix] != 0 : true;
        if (loss_cap) cap = loss_cap[ti.view];
      }
      FwdState st;
      int staged_lo;
      tile_forward<false, NB>(ti, a.n, a.recA, a.recB, a.recC, a.ids, a.rc, s_rec, st, nullptr, s_id,
                          &staged_lo);
      BwdIn in{st.T, ti.inside ? st.last : 0, st.zr, 0.f, 0.f, 0.f, 0.f, 0.f};
      float lpx = 0.f;
      if (ti.inside) {
        const int64_t loc = ti.pix - ti.pix_off;
        const float e0 = st.C0 - tc0, e1 = st.C1 - tc1, e2 = st.C2 - tc2;
        const bool md = m && td > 0.f;
        const float ed = st.D - td;
        if (m) {
          lpx = w_rgb * (fabsf(e0) + fabsf(e1) + fabsf(e2));
          if (md) lpx += w_depth * fabsf(ed);
        }
        if (out.loss) out.loss[ti.pix] = lpx;
        // Outlier pixels (own loss above the view's cap) are ignored.
        const bool keep = m && !(lpx > cap);
        lpx = keep ? lpx : 0.f;
        if (keep) {
          in.sC0 = sgnf(e0);
          in.sC1 = sgnf(e1);
          in.sC2 = sgnf(e2);
          if (md) in.sD = sgnf(ed);
          in.gC0 = w_rgb * in.sC0;
          in.gC1 = w_rgb * in.sC1;
          in.gC2 = w_rgb * in.sC2;
          in.gD = w_depth * in.sD;
        }
        save_state(ps, ti.pix, st);
        if (out.rgb) {
          float *o = out.rgb + 3 * ti.pix_off + loc;
          o[0] = st.C0;
          o[ti.HW] = st.C1;
          o[2 * ti.HW] = st.C2;
        }
        if (out.depth) out.depth[ti.pix] = st.D;
        if (out.T_final) out.T_final[ti.pix] = st.T;
        if (out.last) out.last[ti.pix] = st.last;
      }
      const float ls = wave_sum(lpx);
      if ((threadIdx.x & 63) == 0) s_loss[threadIdx.x >> 6] = ls;
      tile_backward<false>(ti, a.n, a.recA, a.recB, a.recC, a.ids, a.rc, in, grad2d, s_rec, s_part, s_id, &s_max,
                           s_mA, staged_lo, w_rgb, w_depth);
      if (threadIdx.x == 0 && loss) atomicAdd(loss, (s_loss[0] + s_loss[1]) + (s_loss[2] + s_loss[3]));
      if (threadIdx.x == 0) {
        const uint64_t d = wall_clock64() - clk0;
        tile_cost[tile] = d < 0xFFFFFFFFull ? (uint32_t)d : 0xFFFFFFFFu;
        if (blockIdx.x == 0) hdr[HDR_COSTS] = 1u;
      }
      // The next tile may have an empty list (no barrier in its forward):
      // keep its shared-memory writes behind this tile's reads.
      __syncthreads();
    }
  }
}

// Standalone L1 loss gradient for the autograd path (grid.y = view).
__global__ __launch_bounds__(BLOCK) void k_l1(const ViewInfo *__restrict__ views, const float *__restrict__ rgb,
                                              const float *__restrict__ depth,
                                              const float *__restrict__ t_rgb,
                                              const float *__restrict__ t_depth,
                                              const uint8_t *__restrict__ pmask, float w_rgb, float w_depth,
                                              const float *__restrict__ loss_cap,
                                              float *__restrict__ g_rgb, float *__restrict__ g_depth,
                                              float *__restrict__ loss) {
  __shared__ float s_w[4];
  const ViewInfo vi = views[blockIdx.y];
  const int64_t HW = (int64_t)vi.W * vi.H;
  float l = 0.f;
  for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < HW; q += (int64_t)gridDim.x * BLOCK) {
    const int64_t pix = vi.pix_off + q;
    const int64_t c0 = 3 * vi.pix_off + q;
    const bool m0 = pmask ? pmask[pix] != 0 : true;
    const float td = t_depth[pix];
    const float ed = depth[pix] - td;
    float e[3];
    float lp = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      e[ch] = rgb[c0 + ch * HW] - t_rgb[c0 + ch * HW];
      lp += fabsf(e[ch]);
    }
    lp = w_rgb * lp;
    if (td > 0.f) lp += w_depth * fabsf(ed);
    // Outlier pixels (own loss above the view's cap) are ignored.
    const bool m = m0 && !(loss_cap && lp > loss_cap[blockIdx.y]);
    const bool md = m && td > 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) g_rgb[c0 + ch * HW] = m ? w_rgb * sgnf(e[ch]) : 0.f;
    g_depth[pix] = md ? w_depth * sgnf(ed) : 0.f;
    l += m ? lp : 0.f;
  }
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]));
}

void launch_l1(const Plan &p, const ViewInfo *views, const float *rgb, const float *depth,
               const float *t_rgb, const float *t_depth, const uint8_t *pmask, float w_rgb,
               float w_depth, const float *loss_cap, float *g_rgb, float *g_depth, float *loss, hipStream_t s) {
  const unsigned gx = (unsigned)((p.total_pixels / p.n_views + BLOCK - 1) / BLOCK);
  dim3 grid(gx < 1024 ? (gx < 1 ? 1 : gx) : 1024, (unsigned)p.n_views);
  hipLaunchKernelGGL(k_l1, grid, dim3(BLOCK), 0, s, views, rgb, depth, t_rgb, t_depth, pmask, w_rgb, w_depth,
                     loss_cap, g_rgb, g_depth, loss);
}

void launch_render_forward(const Plan &p, const Workspace &ws, const ViewInfo *views,
                           const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                           const gsr_images *out, hipStream_t s) {
  const RasterArgs a = raster_args(ws, views, tile_view, g, rc);
  gsr_images o{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (out) o = *out;
  PixelState ps{ws.T_final, ws.last, ws.zr};
  hipLaunchKernelGGL(k_render_fwd, dim3(p.total_tiles), dim3(BLOCK), 0, s, a, ps, o);
}

void launch_render_backward(const Plan &p, const Workspace &ws, const ViewInfo *views,
                            const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                            const float *g_rgb, const float *g_depth, const float *g_T, hipStream_t s) {
  const RasterArgs a = raster_args(ws, views, tile_view, g, rc);
  hipLaunchKernelGGL(k_render_bwd, dim3(p.total_tiles), dim3(BLOCK), 0, s, a, ws.T_final, ws.last, ws.zr, g_rgb,
                     g_depth, g_T, ws.grad2d);
}

void launch_render_fused(const Plan &p, const Workspace &ws, const ViewInfo *views,
                         const int32_t *tile_view, const gsr_gaussians &g, const RenderConsts &rc,
                         const float *t_rgb, const float *t_depth, const uint8_t *pmask, float w_rgb,
                         float w_depth, const float *loss_cap, const gsr_images *out, float *loss,
                         const Tuning &tun, int num_cus, hipStream_t s) {
  const RasterArgs a = raster_args(ws, views, tile_view, g, rc);
  gsr_images o{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (out) o = *out;
  int grid = tun.blocks_per_cu * num_cus;
  const int need = (p.total_tiles + tun.tiles_per_pop - 1) / tun.tiles_per_pop;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  PixelState ps{nullptr, nullptr, nullptr};  // the fused backward keeps the forward state in registers
  const uint32_t *queue = tun.lpt_order ? ws.queue : nullptr;
#define GSR_LAUNCH_FUSED(NB_)                                                                                  \
  hipLaunchKernelGGL(k_render_fused<NB_>, dim3(grid), dim3(BLOCK), 0, s, a, ws.hdr, queue, p.total_tiles,            \
                     tun.tiles_per_pop, t_rgb, t_depth, pmask, w_rgb, w_depth, loss_cap, o, loss, ws.grad2d, ps,      \
                     ws.tile_cost)
  switch (tun.batch) {
    case 64: GSR_LAUNCH_FUSED(64); break;
    case 128: GSR_LAUNCH_FUSED(128); break;
    case 256: GSR_LAUNCH_FUSED(256); break;
    default: GSR_LAUNCH_FUSED(192); break;
  }
#undef GSR_LAUNCH_FUSED
}

// Totals of the per-pixel work counters: counts[0] pairs, [1] entries the
// forward examined, [2] entries blended, [3] sum of last.
// Work of the last forward, for the roofline: the forward walk of every
// tile again, with counting on and no outputs (the workspace still holds the
// records, lists and ranges of that call).
// The walk also sums every pixel's `last` (the entries the backward walk
// examines) into counts[3], and block 0 copies the pair count into counts[0].
__global__ __launch_bounds__(BLOCK) void k_count_walk(RasterArgs a, const uint32_t *__restrict__ hdr,
                                                      unsigned long long *__restrict__ counts) {
  __shared__ Staged s_rec[BATCH];
  const TileInfo ti = tile_info(blockIdx.x, a.views, a.tile_view, a.ranges);
  FwdState st;
  tile_forward<true>(ti, a.n, a.recA, a.recB, a.recC, a.ids, a.rc, s_rec, st, counts);
  unsigned long long c = ti.inside ? (unsigned long long)st.last : 0ull;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(counts + 3, c);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    counts[0] = *reinterpret_cast<const unsigned long long *>(hdr + HDR_NPAIRS);
}

void launch_work_counts(const Plan &p, const Workspace &ws, const ViewInfo *views, const int32_t *tile_view,
                        const gsr_gaussians &g, const RenderConsts &rc, hipStream_t s) {
  launch_fill_u32(reinterpret_cast<uint32_t *>(ws.counts), 0u, 8, s);
  const RasterArgs a = raster_args(ws, views, tile_view, g, rc);
  if (p.total_tiles > 0)
    hipLaunchKernelGGL(k_count_walk, dim3(p.total_tiles), dim3(BLOCK), 0, s, a, ws.hdr, ws.counts);
}

}  // namespace gsr
