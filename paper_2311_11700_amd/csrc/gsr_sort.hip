// Tile lists: depth sort of the projected Gaussians, emission of
// (tile, Gaussian) pairs in depth order, a stable radix sort of the pairs by
// tile id, and per-tile [start, end) ranges.
//
// The blending order is the lexicographic (tile, float32 depth bits, index)
// order.  A least-significant-digit radix sort of the 64-bit key
// (tile << 32 | depth bits) would make four passes over every pair for the
// depth digits.  All pairs of one Gaussian share its depth, so those four
// passes are run once per Gaussian instead (stable sort of the records by
// depth, ties by record id); the pairs are then emitted in that order and
// only the tile digits are sorted per pair.  The result is identical to the
// 64-bit sort; the pair traffic drops from ceil((32 + tile_bits) / 8) passes
// to ceil(tile_bits / 8).
//
// Every kernel reads its element count from device memory and uses a fixed
// grid, so the whole sequence can be captured in a HIP graph.
#include "gsr_internal.h"

namespace gsr {

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void k_fill_f32(float *__restrict__ p, float v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

static unsigned fill_grid(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

void launch_fill_u32(uint32_t *ptr, uint32_t value, int64_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(count)), dim3(BLOCK), 0, s, ptr, value, count);
}

void launch_fill_f32(float *ptr, float value, int64_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_fill_f32, dim3(fill_grid(count)), dim3(BLOCK), 0, s, ptr, value, count);
}

// Clear the per-call header words (pair count, queue counter).  The overflow
// flag and required count are sticky until gsr_check_overflow reads them; on
// a workspace's first use (no magic yet) they are cleared too.
__global__ void k_reset_header(uint32_t *hdr) {
  if (threadIdx.x == 0) reset_header_words(hdr);
}

void launch_reset_header(const Workspace &ws, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_header, dim3(1), dim3(64), 0, s, ws.hdr);
}

// ----------------------------------------------------------------- block scan

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *s_w, T &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  T pre = 0;
  for (int w = 0; w < wave; ++w) pre += s_w[w];
  total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  __syncthreads();
  return pre + x - v;
}

// ----------------------------------------------------------------- radix sort

__device__ __forceinline__ uint32_t sort_count(const unsigned long long *n_dev, uint32_t n_static,
                                               uint32_t cap) {
  if (!n_dev) return n_static;
  const unsigned long long n = *n_dev;
  return n < cap ? (uint32_t)n : cap;
}

// The last pass of the depth sort carries a weight per key (its record's
// pair count): the histogram also sums the weights per digit and tile, the
// scan scans them, and the scatter gives every output position the
// exclusive prefix of the weights in the sorted order (the record's first
// pair) and fills the emission buckets, so the records need no scan of their
// own before the emission.
struct PassWeights {
  const uint32_t *vals;           // the keys' values (weights are looked up by value)
  const uint32_t *weight;         // weight of the key with value v: weight[v]
  unsigned long long *whist;      // [RADIX][wstride] weight sums per digit and tile
  unsigned long long *whoff;      // [RADIX][wstride] exclusive scan of whist over the tiles
  unsigned long long *wdigit;     // [RADIX] weight totals per digit
  int wstride;
  uint32_t *bucket;               // emission buckets (EMIT_BUCKET pairs each)
  unsigned long long cap;         // pair capacity: offsets are clamped to it
  uint32_t *hdr;                  // pair count and overflow flag
};

// Adds w of every lane in `valid` into acc[d]: one LDS atomic per distinct
// digit of the wavefront (keys of a tile often share their high digits).
__device__ __forceinline__ void wave_add_by_digit(unsigned long long *acc, uint32_t d, unsigned long long w,
                                                  uint64_t valid) {
  const int lane = __lane_id();
  uint64_t todo = valid;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t dl = __shfl(d, leader);
    const uint64_t grp = __ballot(d == dl) & todo;
    unsigned long long x = (grp >> lane) & 1ull ? w : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == leader) atomicAdd(&acc[dl], x);
    todo &= ~grp;
  }
}

// Digit counts of each sort tile (STILE consecutive keys), digit-major (and,
// WEIGHTED, the weight sums).
template <int ITEMS, bool WEIGHTED>
__global__ __launch_bounds__(BLOCK) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                      const unsigned long long *n_dev,
                                                      uint32_t n_static, uint32_t cap, int shift,
                                                      int nbits, uint32_t *__restrict__ hist,
                                                      int max_tiles, PassWeights pw) {
  __shared__ uint32_t cnt[RADIX];
  __shared__ unsigned long long wcnt[WEIGHTED ? RADIX : 1];
  const uint32_t n = sort_count(n_dev, n_static, cap);
  constexpr int STILE = BLOCK * ITEMS;
  const uint32_t ntiles = (n + STILE - 1) / STILE;
  const uint32_t mask = (1u << nbits) - 1u;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    cnt[threadIdx.x] = 0u;
    if (WEIGHTED) wcnt[threadIdx.x] = 0ull;
    uint32_t kr[ITEMS], wr[WEIGHTED ? ITEMS : 1];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const uint32_t idx = t * STILE + r * BLOCK + threadIdx.x;
      kr[r] = idx < n ? keys[idx] : 0u;
      if (WEIGHTED) wr[r] = idx < n ? pw.weight[pw.vals[idx]] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = t * STILE + r * BLOCK + threadIdx.x < n;
      const uint32_t d = (kr[r] >> shift) & mask;
      const uint64_t vmask = __ballot(valid);
      const uint64_t peers = match_digit(d, nbits, vmask);
      if (valid && (peers & lanemask_lt()) == 0ull) atomicAdd(&cnt[d], (uint32_t)__popcll(peers));
      if (WEIGHTED) wave_add_by_digit(wcnt, d, wr[r], vmask);
    }
    __syncthreads();
    // Only the pass's own digits: one scattered word per row and tile.
    if (threadIdx.x <= mask) {
      hist[(size_t)threadIdx.x * max_tiles + t] = cnt[threadIdx.x];
      if (WEIGHTED) pw.whist[(size_t)threadIdx.x * pw.wstride + t] = wcnt[threadIdx.x];
    }
    __syncthreads();
  }
}

// One block per digit: exclusive scan over the tiles of that digit's column
// (counts stay in hist, offsets go to hoff; WEIGHTED, the same for the
// weight sums).
template <int ITEMS, bool WEIGHTED>
__global__ __launch_bounds__(BLOCK) void k_radix_scan(const uint32_t *__restrict__ hist,
                                                      uint32_t *__restrict__ hoff,
                                                      const unsigned long long *n_dev,
                                                      uint32_t n_static, uint32_t cap, int max_tiles,
                                                      uint32_t *__restrict__ digit_total, PassWeights pw) {
  __shared__ uint32_t s_w[4];
  __shared__ unsigned long long s_w64[4];
  const uint32_t n = sort_count(n_dev, n_static, cap);
  constexpr int STILE = BLOCK * ITEMS;
  const uint32_t ntiles = (n + STILE - 1) / STILE;
  const uint32_t *col = hist + (size_t)blockIdx.x * max_tiles;
  uint32_t *ocol = hoff + (size_t)blockIdx.x * max_tiles;
  uint32_t carry = 0u;
  for (uint32_t base = 0; base < ntiles; base += BLOCK * SCAN_ITEMS) {
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0u;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const uint32_t idx = base + threadIdx.x * SCAN_ITEMS + k;
      v[k] = idx < ntiles ? col[idx] : 0u;
      sum += v[k];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan<uint32_t>(sum, s_w, total) + carry;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const uint32_t idx = base + threadIdx.x * SCAN_ITEMS + k;
      if (idx < ntiles) ocol[idx] = pre;
      pre += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
  if (WEIGHTED) {
    const unsigned long long *wcol = pw.whist + (size_t)blockIdx.x * pw.wstride;
    unsigned long long *wocol = pw.whoff + (size_t)blockIdx.x * pw.wstride;
    unsigned long long wcarry = 0ull;
    for (uint32_t base = 0; base < ntiles; base += BLOCK * SCAN_ITEMS) {
      unsigned long long v[SCAN_ITEMS];
      unsigned long long sum = 0ull;
#pragma unroll
      for (int k = 0; k < SCAN_ITEMS; ++k) {
        const uint32_t idx = base + threadIdx.x * SCAN_ITEMS + k;
        v[k] = idx < ntiles ? wcol[idx] : 0ull;
        sum += v[k];
      }
      unsigned long long total;
      unsigned long long pre = block_exclusive_scan<unsigned long long>(sum, s_w64, total) + wcarry;
#pragma unroll
      for (int k = 0; k < SCAN_ITEMS; ++k) {
        const uint32_t idx = base + threadIdx.x * SCAN_ITEMS + k;
        if (idx < ntiles) wocol[idx] = pre;
        pre += v[k];
      }
      wcarry += total;
    }
    if (threadIdx.x == 0) pw.wdigit[blockIdx.x] = wcarry;
  }
}

// Stable scatter of one digit pass.  Wavefront w ranks the w-th quarter of
// the sort tile: equal digits inside a row of 64 keys by ballot matching, and
// across its rows by wavefront-private counts per digit in LDS (no block
// barrier between rows).  The per-wavefront counts, the tile's digit counts
// and the digit offsets then place every key in block-local digit order in
// LDS, and each digit's keys of the tile are written as one contiguous run:
// consecutive threads store consecutive addresses.
//
// With tile_count, sort tile t holds only its first tile_count[t] keys (the
// rest of its slots are unused).  With key_limit != 0, keys >= key_limit are
// left out (the digit counts in hist must leave them out too).  The output
// is dense either way; with n_out, block 0 stores the number of keys
// written there.
//
// WEIGHTED (the depth sort's last pass): keys_out receives, instead of the
// keys, each position's exclusive prefix of the weights in the sorted order
// clamped to the capacity, every emission bucket b gets the position holding
// weight unit EMIT_BUCKET b (and the one after the last bucket the position
// holding the last emitted unit), and block 0 stores the weight total as the
// pair count (with the overflow flag when it exceeds the capacity).
template <int ITEMS, bool VALS, bool WEIGHTED>
__global__ __launch_bounds__(BLOCK) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const unsigned long long *n_dev, uint32_t n_static, uint32_t cap, int shift, int nbits,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ hoff, int max_tiles,
    const uint32_t *__restrict__ digit_total, const uint32_t *__restrict__ tile_count,
    uint32_t key_limit, unsigned long long *__restrict__ n_out, PassWeights pw) {
  static_assert(!WEIGHTED || VALS, "weights are looked up by value");
  constexpr int STILE = BLOCK * ITEMS;
  constexpr int WKEYS = 64 * ITEMS;
  __shared__ unsigned long long s_wbase[WEIGHTED ? RADIX : 1];  // weight before each digit
  __shared__ unsigned long long s_wgoff[WEIGHTED ? RADIX : 1];  // weight before the tile's run of each digit
  __shared__ unsigned long long s_lw[WEIGHTED ? RADIX : 1];     // local weight before each digit's run
  __shared__ unsigned long long s_w64[4];
  __shared__ uint32_t s_c[WEIGHTED ? STILE : 1];                // weight of each local slot
  __shared__ unsigned long long s_e[WEIGHTED ? STILE : 1];      // exclusive weight prefix over the local slots
  __shared__ unsigned long long s_wtotal;
  __shared__ uint32_t s_base[RADIX];   // first output position of each digit
  __shared__ uint32_t s_goff[RADIX];   // output position minus local position, per digit
  __shared__ uint32_t s_lbase[RADIX];  // first local position of each digit
  __shared__ uint32_t s_wc[4][RADIX];  // per-wavefront digit counts, then their prefix over wavefronts
  __shared__ uint32_t s_w[4];
  __shared__ uint32_t s_k[STILE];
  __shared__ uint32_t s_v[VALS ? STILE : 1];
  const uint32_t n = sort_count(n_dev, n_static, cap);
  const uint32_t ntiles = (n + STILE - 1) / STILE;
  const uint32_t mask = (1u << nbits) - 1u;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int dig = threadIdx.x;
  {
    uint32_t total;
    s_base[dig] = block_exclusive_scan<uint32_t>(dig <= (int)mask ? digit_total[dig] : 0u, s_w, total);
    if (n_out && blockIdx.x == 0 && threadIdx.x == 0) *n_out = total;
  }
  if (WEIGHTED) {
    unsigned long long wtotal;
    s_wbase[dig] = block_exclusive_scan<unsigned long long>(dig <= (int)mask ? pw.wdigit[dig] : 0ull, s_w64, wtotal);
    if (threadIdx.x == 0) s_wtotal = wtotal;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *reinterpret_cast<unsigned long long *>(pw.hdr + HDR_NPAIRS) = wtotal;
      if (wtotal > pw.cap) {
        atomicOr(pw.hdr + HDR_OVERFLOW, 1u);
        atomicMax(reinterpret_cast<unsigned long long *>(pw.hdr + HDR_REQUIRED), wtotal);
      }
    }
  }
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t t0 = t * STILE;
    const uint32_t tn = tile_count ? tile_count[t] : (n - t0 < (uint32_t)STILE ? n - t0 : (uint32_t)STILE);
    const uint32_t tend = t0 + tn;  // keys of this tile: [t0, tend)
    const uint32_t wbase = t0 + wave * WKEYS + lane;
    uint32_t kr[ITEMS], vr[ITEMS], rank[ITEMS], cr[WEIGHTED ? ITEMS : 1];
    uint32_t live = 0u;  // bit r: item r is a key to sort
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const uint32_t idx = wbase + r * 64;
      kr[r] = idx < tend ? keys_in[idx] : 0u;
      if (VALS) vr[r] = idx < tend ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (wbase + r * 64 < tend && (key_limit == 0u || kr[r] < key_limit)) live |= 1u << r;
    if (WEIGHTED) {
#pragma unroll
      for (int r = 0; r < ITEMS; ++r) cr[r] = (live >> r) & 1u ? pw.weight[vr[r]] : 0u;
    }
    s_wc[0][dig] = s_wc[1][dig] = s_wc[2][dig] = s_wc[3][dig] = 0u;
    uint32_t tkeys;  // keys of this tile that are sorted (block-uniform)
    {
      const bool used = dig <= (int)mask;  // rows past the pass's digits are not stored
      const uint32_t cnt = used ? hist[(size_t)dig * max_tiles + t] : 0u;
      const uint32_t lbase = block_exclusive_scan<uint32_t>(cnt, s_w, tkeys);
      s_lbase[dig] = lbase;
      s_goff[dig] = s_base[dig] + (used ? hoff[(size_t)dig * max_tiles + t] : 0u) - lbase;
    }
    if (WEIGHTED) {
      unsigned long long ltot;
      const bool used = dig <= (int)mask;
      s_lw[dig] = block_exclusive_scan<unsigned long long>(used ? pw.whist[(size_t)dig * pw.wstride + t] : 0ull,
                                                           s_w64, ltot);
      s_wgoff[dig] = s_wbase[dig] + (used ? pw.whoff[(size_t)dig * pw.wstride + t] : 0ull);
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = (live >> r) & 1u;
      const uint32_t d = (kr[r] >> shift) & mask;
      const uint64_t peers = match_digit(d, nbits, __ballot(valid));
      const uint64_t below = peers & lanemask_lt();
      // Wavefront-private counts: every lane reads before the group's
      // leader adds the group size (program order within the wavefront).
      const uint32_t before = valid ? s_wc[wave][d] : 0u;
      rank[r] = before + (uint32_t)__popcll(below);
      if (valid && below == 0ull) s_wc[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
      const uint32_t c0 = s_wc[0][dig], c1 = s_wc[1][dig], c2 = s_wc[2][dig];
      s_wc[0][dig] = s_lbase[dig];
      s_wc[1][dig] = s_lbase[dig] + c0;
      s_wc[2][dig] = s_lbase[dig] + c0 + c1;
      s_wc[3][dig] = s_lbase[dig] + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      if ((live >> r) & 1u) {
        const uint32_t lp = s_wc[wave][(kr[r] >> shift) & mask] + rank[r];
        s_k[lp] = kr[r];
        if (VALS) s_v[lp] = vr[r];
        if (WEIGHTED) s_c[lp] = cr[r];
      }
    }
    __syncthreads();
    if (WEIGHTED) {
      // Exclusive prefix of the weights over the local slots (thread t:
      // slots [t ITEMS, (t + 1) ITEMS)).
      const uint32_t s0 = threadIdx.x * (uint32_t)ITEMS;
      unsigned long long sum = 0ull;
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) sum += s0 + q < tkeys ? s_c[s0 + q] : 0u;
      unsigned long long ltot;
      unsigned long long pre = block_exclusive_scan<unsigned long long>(sum, s_w64, ltot);
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        if (s0 + q < tkeys) {
          s_e[s0 + q] = pre;
          pre += s_c[s0 + q];
        }
      }
      __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < tkeys; i += BLOCK) {
      const uint32_t key = s_k[i];
      const uint32_t d = (key >> shift) & mask;
      const uint32_t gpos = s_goff[d] + i;
      if (!WEIGHTED) {
        keys_out[gpos] = key;
      } else {
        // The record's first pair and the emission buckets it holds.
        const unsigned long long o = s_wgoff[d] + (s_e[i] - s_lw[d]);
        const unsigned long long oe = o + s_c[i];
        const unsigned long long e = oe < pw.cap ? oe : pw.cap;
        const unsigned long long n_emit = s_wtotal < pw.cap ? s_wtotal : pw.cap;
        keys_out[gpos] = (uint32_t)(o < pw.cap ? o : pw.cap);
        for (unsigned long long b = (o + EMIT_BUCKET - 1) / EMIT_BUCKET; b * EMIT_BUCKET < e; ++b)
          pw.bucket[b] = gpos;
        if (o < n_emit && n_emit <= e) pw.bucket[(n_emit + EMIT_BUCKET - 1) / EMIT_BUCKET] = gpos;
      }
      if (VALS) vals_out[gpos] = s_v[i];
    }
    __syncthreads();
  }
}

// Stable LSD radix sort of (key, value) over bits [0, key_bits); returns the
// index of the buffer holding the result.
// The key occupies bits [base, base + key_bits) of each word; without vals
// the words are sorted alone (packed pairs).  When hist0_ready, the first
// pass's per-tile digit counts are already in hist (written by the kernel
// that produced the keys).
//
// With tile_count0, the first pass reads tile t's first tile_count0[t] keys
// only (n_static covering all tiles' slots); with key_limit0 != 0 it drops the
// words >= key_limit0 (the hist0_ready counts leave them out).  With
// n_after0, the first pass stores the number of words it kept there and the
// later passes sort that many.  With wlast, the last pass is weighted (see
// PassWeights; wlast->vals is filled in here).
template <int ITEMS>
static int radix_sort(uint32_t *keys[2], uint32_t *vals[2], const unsigned long long *n_dev,
                      uint32_t n_static, uint32_t cap, int base, int key_bits, uint32_t *hist, uint32_t *hoff,
                      int max_tiles, uint32_t *digit_total, int grid, bool hist0_ready,
                      const uint32_t *tile_count0, uint32_t key_limit0, unsigned long long *n_after0,
                      const PassWeights *wlast, hipStream_t s) {
  const int per = radix_digit_bits(key_bits);
  int cur = 0;
  for (int sh = 0; sh < key_bits; sh += per) {
    const int nbits = key_bits - sh < per ? key_bits - sh : per;
    const int shift = base + sh;
    const bool weighted = wlast && sh + per >= key_bits;
    PassWeights pw{};
    if (weighted) {
      pw = *wlast;
      pw.vals = vals[cur];
    }
    const uint32_t *tile_count = sh == 0 ? tile_count0 : nullptr;
    const uint32_t key_limit = sh == 0 ? key_limit0 : 0u;
    unsigned long long *n_out = sh == 0 ? n_after0 : nullptr;
    if (sh > 0 && n_after0) n_dev = n_after0;
    if (sh > 0 || !hist0_ready) {
      if (weighted)
        hipLaunchKernelGGL((k_radix_hist<ITEMS, true>), dim3(grid), dim3(BLOCK), 0, s, keys[cur], n_dev, n_static,
                           cap, shift, nbits, hist, max_tiles, pw);
      else
        hipLaunchKernelGGL((k_radix_hist<ITEMS, false>), dim3(grid), dim3(BLOCK), 0, s, keys[cur], n_dev,
                           n_static, cap, shift, nbits, hist, max_tiles, pw);
    }
    if (weighted)
      hipLaunchKernelGGL((k_radix_scan<ITEMS, true>), dim3(1u << nbits), dim3(BLOCK), 0, s, hist, hoff, n_dev, n_static,
                         cap, max_tiles, digit_total, pw);
    else
      hipLaunchKernelGGL((k_radix_scan<ITEMS, false>), dim3(1u << nbits), dim3(BLOCK), 0, s, hist, hoff, n_dev,
                         n_static, cap, max_tiles, digit_total, pw);
    if (weighted)
      hipLaunchKernelGGL((k_radix_scatter<ITEMS, true, true>), dim3(grid), dim3(BLOCK), 0, s, keys[cur],
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_dev, n_static, cap, shift, nbits, hist, hoff,
                         max_tiles, digit_total, tile_count, key_limit, n_out, pw);
    else if (vals)
      hipLaunchKernelGGL((k_radix_scatter<ITEMS, true, false>), dim3(grid), dim3(BLOCK), 0, s, keys[cur],
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_dev, n_static, cap, shift, nbits, hist, hoff,
                         max_tiles, digit_total, tile_count, key_limit, n_out, pw);
    else
      hipLaunchKernelGGL((k_radix_scatter<ITEMS, false, false>), dim3(grid), dim3(BLOCK), 0, s, keys[cur],
                         (const uint32_t *)nullptr, keys[cur ^ 1], (uint32_t *)nullptr, n_dev, n_static, cap,
                         shift, nbits, hist, hoff, max_tiles, digit_total, tile_count, key_limit, n_out, pw);
    cur ^= 1;
  }
  return cur;
}

static int sort_grid_for(int64_t n, int items, int cap_grid) {
  int64_t t = (n + (int64_t)BLOCK * items - 1) / ((int64_t)BLOCK * items);
  if (t > cap_grid) t = cap_grid;
  return t < 1 ? 1 : (int)t;
}

// Only the visible records (compacted per tile by the projection) are
// sorted; their number is known after the first pass.  The last pass is
// weighted by the records' pair counts: dvals[dsorted] gets the record
// order, dkeys[dsorted] each record's first pair (clamped to the capacity),
// bucket_rec the emission buckets, and the header the pair count.
int launch_depth_sort(const Plan &p, Workspace &ws, hipStream_t s, int sort_grid) {
  unsigned long long *n_vis = reinterpret_cast<unsigned long long *>(ws.hdr + HDR_NVISIBLE);
  PassWeights w{};
  w.weight = ws.count;
  w.whist = ws.whist;
  w.whoff = ws.whoff;
  w.wdigit = ws.wdigit;
  w.wstride = p.depth_tiles;
  w.bucket = ws.bucket_rec;
  w.cap = (unsigned long long)p.capacity;
  w.hdr = ws.hdr;
  ws.dsorted = radix_sort<SORT_ITEMS_DEPTH>(ws.dkeys, ws.dvals, nullptr, (uint32_t)p.n_rec, (uint32_t)p.n_rec, 0, 32,
                                            ws.hist, ws.hoff, p.max_sort_tiles, ws.digit_total,
                                            sort_grid_for(p.n_rec, SORT_ITEMS_DEPTH, sort_grid), true,
                                            ws.tile_visible, 0u, n_vis, &w, s);
  return ws.dsorted;
}

// The first pass drops the pairs outside the alpha support (tile key
// total_tiles, left out of the emission's digit counts): the later passes,
// the tile ranges and the lists see only the listed pairs, whose number goes
// to the header.
int launch_pair_sort(const Plan &p, Workspace &ws, hipStream_t s, int sort_grid) {
  const unsigned long long *n_dev = reinterpret_cast<const unsigned long long *>(ws.hdr + HDR_NPAIRS);
  unsigned long long *n_listed = reinterpret_cast<unsigned long long *>(ws.hdr + HDR_NLISTED);
  const uint32_t key_limit = (uint32_t)p.total_tiles << ws.pack_shift;
  ws.psorted = radix_sort<SORT_ITEMS_PAIR>(ws.pkeys, ws.pack_shift ? nullptr : ws.pvals, n_dev, 0u,
                                           (uint32_t)p.capacity, ws.pack_shift, p.tile_bits,
                                           ws.hist, ws.hoff, p.max_sort_tiles, ws.digit_total,
                                           sort_grid_for(p.capacity, SORT_ITEMS_PAIR, sort_grid), true, nullptr,
                                           key_limit, n_listed, nullptr, s);
  return ws.psorted;
}

// ------------------------------------------------------------------ emit pairs

// Pair emission.  A block-iteration produces one sort tile of the pair sort
// (STILE consecutive pairs, in depth order): the records that own those pairs
// (found through the bucket index) are staged in LDS, up to EMIT_STAGE at a time,
// with their pair offsets, rectangles, alpha-support parameters and conics;
// then one thread per pair finds its record among the staged ones, decodes
// the tile from the rectangle, tests it against the alpha support and writes
// the word(s).  The block also counts the first radix pass's digits of its
// tile.  Global loads come in two dependent rounds per staged chunk of
// records instead of per pair.
//
// Staged records are consecutive and each holds at least one pair, so the
// staged record of pair p is the last one starting at or before p: every
// staged record writes its index at its first pair in an LDS map of the
// chunk's pairs, and a block-wide running maximum over the map fills in the
// rest (one LDS read per pair afterwards).
//
// The alpha-support test of a record with the cull bit depends only on the
// row: after staging, the block evaluates the row ranges of all its staged
// records once (one row per thread, spread evenly over the block; up to
// EMIT_ROWS rows, the rest per pair) and every pair looks its row up.
constexpr int EMIT_ROWS = 1024;
// Records staged per round: with the block's LDS at 21 KB and its registers
// held to seven wavefronts per SIMD, seven blocks share a CU, which hides the
// staging gathers' latency better than four blocks staging a full BLOCK of
// records each.
constexpr int EMIT_STAGE = 128;
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(7))) void k_emit_pairs(const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ off,
                                                      const uint4 *__restrict__ tinfo,
                                                      const Support *__restrict__ support,
                                                      const float4 *__restrict__ recB, uint32_t dropped_key,
                                                      const unsigned long long *__restrict__ n_vis,
                                                      const unsigned long long *__restrict__ n_dev,
                                                      uint32_t cap, const uint32_t *__restrict__ bucket_rec,
                                                      uint32_t *__restrict__ pkeys, uint32_t *__restrict__ pvals,
                                                      int pack_shift, int nbits0, uint32_t *__restrict__ hist,
                                                      int max_tiles) {
  static_assert(EMIT_BUCKET == BLOCK, "one emission bucket per BLOCK pairs");
  constexpr int STILE = BLOCK * SORT_ITEMS_PAIR;
  __shared__ uint32_t s_off[EMIT_STAGE + 1];  // first pair of each staged record, then the end
  __shared__ uint32_t s_id[EMIT_STAGE];
  __shared__ uint4 s_ti[EMIT_STAGE];
  __shared__ Support s_sp[EMIT_STAGE];
  __shared__ float4 s_cb[EMIT_STAGE];
  __shared__ uint32_t s_cnt[RADIX];
  __shared__ uint16_t s_map[STILE];             // staged record of each pair of the chunk (pair - p0)
  __shared__ uint32_t s_rbase[EMIT_STAGE];      // first row slot of each staged record (culled records' rows)
  __shared__ uint32_t s_row[EMIT_ROWS];         // column range of a row: first | count << 16
  __shared__ uint32_t s_w[4];
  const uint32_t n = sort_count(n_dev, 0u, cap);
  const uint32_t n_rec = (uint32_t)*n_vis;  // depth-ordered records
  const uint32_t ntiles = (n + STILE - 1) / STILE;
  const uint32_t mask0 = (1u << nbits0) - 1u;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  for (uint32_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    const uint32_t p0 = T * STILE;
    const uint32_t p1 = p0 + STILE < n ? p0 + STILE : n;
    // Records holding pairs p0 .. p1 - 1: from the one holding p0 (a bucket
    // start) to the one holding the next tile's first pair (or the last).
    const uint32_t r_first = bucket_rec[p0 / EMIT_BUCKET];
    const uint32_t r_last = bucket_rec[(p1 + EMIT_BUCKET - 1) / EMIT_BUCKET];
    s_cnt[t] = 0u;
    for (uint32_t rb = r_first; rb <= r_last; rb += EMIT_STAGE) {
      const uint32_t nr = r_last - rb + 1u < (uint32_t)EMIT_STAGE ? r_last - rb + 1u : (uint32_t)EMIT_STAGE;
      __syncthreads();
      uint32_t rows = 0u;  // rows of this thread's staged record that need the support test
      if ((uint32_t)t < nr) {
        const uint32_t k = rb + t;
        const uint32_t rec = order[k];
        s_off[t] = off[k];
        s_id[t] = rec;
        const uint4 ti = tinfo[rec];
        s_ti[t] = ti;
        if (ti.y & 0x80000000u) {  // only the culled records use the support and the conic
          s_sp[t] = support[rec];
          s_cb[t] = recB[rec];
          rows = (ti.w >> 16) - (ti.w & 0xFFFFu) + 1u;
        }
      }
      if (t == 0) s_off[nr] = rb + nr < n_rec ? off[rb + nr] : n;
      uint32_t rows_total;
      {
        const uint32_t rb0 = block_exclusive_scan<uint32_t>(rows, s_w, rows_total);
        if (t < EMIT_STAGE) s_rbase[t] = rb0;
      }
      __syncthreads();
      // Row ranges: slot i belongs to the last staged record whose first slot
      // is <= i (records without rows share the next one's first slot).
      const uint32_t rows_cached = rows_total < (uint32_t)EMIT_ROWS ? rows_total : (uint32_t)EMIT_ROWS;
      for (uint32_t i = (uint32_t)t; i < rows_cached; i += BLOCK) {
        int lo = 0, hi = (int)nr - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rbase[mid] <= i) lo = mid;
          else hi = mid - 1;
        }
        const uint4 ti = s_ti[lo];
        const float4 cb = s_cb[lo];
        const int ty = (int)(ti.w & 0xFFFFu) + (int)(i - s_rbase[lo]);
        int c0 = 0;
        const int len = support_row(s_sp[lo], (double)cb.x, (double)cb.y, (double)cb.z, ty, (int)(ti.z & 0xFFFFu),
                                    (int)(ti.z >> 16), c0);
        s_row[i] = (uint32_t)c0 | (uint32_t)len << 16;
      }
      __syncthreads();
      const uint32_t q0 = s_off[0] > p0 ? s_off[0] : p0;
      const uint32_t q1 = s_off[nr] < p1 ? s_off[nr] : p1;
      // Pair -> staged record over [q0, q1) (map index pair - p0): record
      // starts, then a running maximum (thread t: SORT_ITEMS_PAIR consecutive
      // entries of the chunk's STILE).
      {
        const uint32_t e0 = (uint32_t)t * SORT_ITEMS_PAIR;
#pragma unroll
        for (int k = 0; k < SORT_ITEMS_PAIR; ++k) s_map[e0 + k] = 0;
        __syncthreads();
        if ((uint32_t)t < nr && s_off[t] > q0 && s_off[t] < q1) s_map[s_off[t] - p0] = (uint16_t)t;
        __syncthreads();
        uint32_t v[SORT_ITEMS_PAIR], run = 0u;
#pragma unroll
        for (int k = 0; k < SORT_ITEMS_PAIR; ++k) {
          run = max(run, (uint32_t)s_map[e0 + k]);
          v[k] = run;
        }
        // Inclusive running maximum of the threads' last values.
        uint32_t x = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(x, o);
          if (lane >= o) x = max(x, y);
        }
        if (lane == 63) s_w[wv] = x;
        __syncthreads();
        uint32_t before = __shfl_up(x, 1);
        if (lane == 0) before = 0u;
        for (int w = 0; w < wv; ++w) before = max(before, s_w[w]);
#pragma unroll
        for (int k = 0; k < SORT_ITEMS_PAIR; ++k) s_map[e0 + k] = (uint16_t)max(v[k], before);
        __syncthreads();
      }
      for (uint32_t base = q0; base < q1; base += BLOCK) {
        const uint32_t p = base + (uint32_t)t;
        const bool valid = p < q1;
        uint32_t tile = 0u;
        if (valid) {
          const uint32_t a = s_map[p - p0];
          const uint32_t j = p - s_off[a];
          const uint4 ti = s_ti[a];
          const int TX = (int)(ti.y & 0x7FFFFFFFu);
          const int tx0 = (int)(ti.z & 0xFFFFu), tx1 = (int)(ti.z >> 16);
          const int ty0 = (int)(ti.w & 0xFFFFu);
          const uint32_t w = (uint32_t)(tx1 - tx0 + 1);
          // j < 2^24 and w < 2^16: the float quotient is within one of the
          // integer quotient; fix it up exactly.
          uint32_t q = (uint32_t)((float)j / (float)w);
          if (q * w > j) --q;
          else if ((q + 1u) * w <= j) ++q;
          const int ty = ty0 + (int)q, tx = tx0 + (int)(j - q * w);
          tile = ti.x + (uint32_t)(ty * TX + tx);
          if (ti.y & 0x80000000u) {
            // Tiles of the rectangle that the alpha support does not reach
            // get the key past the last tile: the pair sort's first pass
            // drops them.
            const uint32_t slot = s_rbase[a] + q;
            int c0 = 0, len;
            if (slot < (uint32_t)EMIT_ROWS) {
              const uint32_t v = s_row[slot];
              c0 = (int)(v & 0xFFFFu);
              len = (int)(v >> 16);
            } else {
              const float4 cb = s_cb[a];
              len = support_row(s_sp[a], (double)cb.x, (double)cb.y, (double)cb.z, ty, tx0, tx1, c0);
            }
            if (tx < c0 || tx >= c0 + len) tile = dropped_key;
          }
          const uint32_t rec = s_id[a];
          if (pvals) {
            pkeys[p] = tile;
            pvals[p] = rec;
          } else {
            pkeys[p] = tile << pack_shift | rec;
          }
        }
        // The first pass's digit counts leave the dropped pairs out.  The
        // pairs of a row of a rectangle have consecutive tiles, so the lanes
        // of a wavefront rarely share a digit: one LDS atomic per lane.
        if (valid && tile != dropped_key) atomicAdd(&s_cnt[tile & mask0], 1u);
      }
    }
    __syncthreads();
    if (t <= (int)mask0) hist[(size_t)t * max_tiles + T] = s_cnt[t];
  }
}

void launch_emit_pairs(const Plan &p, const Workspace &ws, const ViewInfo *views, hipStream_t s) {
  (void)views;
  const uint32_t *order = ws.dvals[ws.dsorted];
  const uint32_t *off = ws.dkeys[ws.dsorted];  // first pair of each record (the depth sort's last pass)
  const unsigned long long *n_vis = reinterpret_cast<const unsigned long long *>(ws.hdr + HDR_NVISIBLE);
  int64_t blocks = (p.capacity + (int64_t)BLOCK * SORT_ITEMS_PAIR - 1) / ((int64_t)BLOCK * SORT_ITEMS_PAIR);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const unsigned long long *n_dev = reinterpret_cast<const unsigned long long *>(ws.hdr + HDR_NPAIRS);
  hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)blocks), dim3(BLOCK), 0, s, order, off, ws.tinfo, ws.support,
                     ws.recB, (uint32_t)p.total_tiles, n_vis, n_dev, (uint32_t)p.capacity,
                     ws.bucket_rec, ws.pkeys[0], ws.pack_shift ? nullptr : ws.pvals[0], ws.pack_shift,
                     radix_digit_bits(p.tile_bits), ws.hist,
                     p.max_sort_tiles);
}

// ---------------------------------------------------------------- tile ranges

// Every tile's [start, end) in the sorted words, each written once: at a
// change of tile between positions i - 1 and i, the thread of position i
// closes the earlier tile, writes (i, i) for the empty tiles in between and
// opens the later one; the last position closes its tile and empties the
// rest.  Keys past the last tile open nothing (the pair sort has already
// dropped the pairs outside the alpha support).
__global__ __launch_bounds__(BLOCK) void k_tile_ranges(const uint32_t *__restrict__ keys,
                                                       const unsigned long long *n_dev, uint32_t cap,
                                                       uint32_t total_tiles, int shift,
                                                       int2 *__restrict__ ranges) {
  const uint32_t n = sort_count(n_dev, 0u, cap);
  const int64_t T = total_tiles;
  if (n == 0u) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < T; t += (int64_t)gridDim.x * BLOCK)
      ranges[t] = make_int2(0, 0);
    return;
  }
  for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    const int64_t t = (int64_t)(keys[i] >> shift);
    const int64_t tp = i == 0u ? -1 : (int64_t)(keys[i - 1] >> shift);
    if (t != tp) {
      if (tp >= 0 && tp < T) ranges[tp].y = (int)i;
      for (int64_t e = tp + 1; e < t && e < T; ++e) ranges[e] = make_int2((int)i, (int)i);
      if (t < T) ranges[t].x = (int)i;
    }
    if (i + 1u == n) {
      if (t < T) ranges[t].y = (int)n;
      for (int64_t e = t + 1; e < T; ++e) ranges[e] = make_int2((int)n, (int)n);
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_unpack_ids(const uint32_t *__restrict__ words,
                                                      const unsigned long long *n_dev, uint32_t cap,
                                                      uint32_t mask, uint32_t *__restrict__ ids) {
  const uint32_t n = sort_count(n_dev, 0u, cap);
  for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) ids[i] = words[i] & mask;
}

void launch_unpack_ids(const Plan &p, const Workspace &ws, hipStream_t s) {
  const unsigned long long *n_dev = reinterpret_cast<const unsigned long long *>(ws.hdr + HDR_NLISTED);
  hipLaunchKernelGGL(k_unpack_ids, dim3(1024), dim3(BLOCK), 0, s, ws.pkeys[ws.psorted], n_dev,
                     (uint32_t)p.capacity, ws.id_mask, ws.pvals[ws.psorted]);
}

void launch_tile_ranges(const Plan &p, const Workspace &ws, hipStream_t s) {
  const unsigned long long *n_dev = reinterpret_cast<const unsigned long long *>(ws.hdr + HDR_NLISTED);
  int64_t blocks = (p.capacity + BLOCK - 1) / BLOCK;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)blocks), dim3(BLOCK), 0, s, ws.pkeys[ws.psorted],
                     n_dev, (uint32_t)p.capacity, (uint32_t)p.total_tiles, ws.pack_shift, ws.ranges);
}

// ------------------------------------------------------- work order

// The rasteriser's work order as a kernel of its own (one block): used where
// the projection does not write it (no Gaussians; the autotuner's trials).
constexpr int QUEUE_BLOCK = 1024;

__global__ __launch_bounds__(QUEUE_BLOCK) void k_queue_order(const uint32_t *__restrict__ tile_cost,
                                                             const uint32_t *__restrict__ hdr, int total,
                                                             uint32_t *__restrict__ queue) {
  __shared__ uint32_t s_cnt[RADIX];
  __shared__ uint32_t s_cur[RADIX];
  __shared__ uint32_t s_w[QUEUE_BLOCK / 64];
  order_tiles<QUEUE_BLOCK>(tile_cost, hdr[HDR_COSTS] != 0u, total, queue, s_cnt, s_cur, s_w);
}

void launch_queue_order(const Workspace &ws, int total_tiles, hipStream_t s) {
  if (total_tiles > 0)
    hipLaunchKernelGGL(k_queue_order, dim3(1), dim3(QUEUE_BLOCK), 0, s, ws.tile_cost, ws.hdr, total_tiles,
                       ws.queue);
}

}  // namespace gsr
