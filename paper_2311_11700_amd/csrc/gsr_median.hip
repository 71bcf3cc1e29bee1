// Loss cap of the tracking loss: factor x the lower median of every view's
// per-pixel loss (the paper's implementation details drop tracking pixels
// whose loss exceeds ten times the median).  Exact radix select on the float
// bit patterns, one block per view: three histogram passes over 11, 11 and
// 10 bits, each narrowing the candidates to the bin that holds the rank.
#include <math.h>

#include "gsr_internal.h"

namespace gsr {

constexpr int MED_BLOCK = 1024;
constexpr int MED_WAVES = MED_BLOCK / 64;

// Order key of a loss value: non-negative floats order like their bit
// patterns; negative values and -0 count as 0, NaN sorts above +inf.
__device__ __forceinline__ uint32_t loss_key(float v) {
  const uint32_t b = __float_as_uint(v);
  const uint32_t a = b & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return a;  // NaN of either sign
  return (b & 0x80000000u) ? 0u : b;
}

// Exclusive scan of one value per thread over the 1024-thread block; the
// block total goes to *total.
__device__ __forceinline__ uint32_t med_block_scan(uint32_t v, uint32_t *s_w, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint32_t w = lane < MED_WAVES ? s_w[lane] : 0u;
    for (int o = 1; o < MED_WAVES; o <<= 1) {
      const uint32_t y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < MED_WAVES) s_w[lane] = w;  // inclusive wave prefix
  }
  __syncthreads();
  const uint32_t before = wave > 0 ? s_w[wave - 1] : 0u;
  *total = s_w[MED_WAVES - 1];
  return before + x - v;
}

__global__ __launch_bounds__(MED_BLOCK) void k_loss_median(const ViewInfo *__restrict__ views,
                                                           const float *__restrict__ px_loss,
                                                           const uint8_t *__restrict__ pmask, float factor,
                                                           float *__restrict__ cap_out) {
  __shared__ uint32_t hist[2 * MED_BLOCK];
  __shared__ uint32_t s_w[MED_WAVES];
  __shared__ uint32_t s_sel[2];
  const ViewInfo vi = views[blockIdx.x];
  const int64_t HW = (int64_t)vi.W * vi.H;
  const float *L = px_loss + vi.pix_off;
  const uint8_t *M = pmask ? pmask + vi.pix_off : nullptr;
  constexpr int shift[3] = {21, 10, 0};
  constexpr int width[3] = {11, 11, 10};
  uint32_t prefix = 0, k = 0;
  for (int pass = 0; pass < 3; ++pass) {
    const int sh = shift[pass];
    const uint32_t digit_mask = (1u << width[pass]) - 1u;
    const int hi = sh + width[pass];
    hist[threadIdx.x] = 0u;
    hist[threadIdx.x + MED_BLOCK] = 0u;
    __syncthreads();
    for (int64_t q = threadIdx.x; q < HW; q += MED_BLOCK) {
      if (M && M[q] == 0) continue;
      const uint32_t key = loss_key(L[q]);
      if (pass > 0 && (key >> hi) != prefix) continue;
      atomicAdd(&hist[(key >> sh) & digit_mask], 1u);
    }
    __syncthreads();
    const uint32_t c0 = hist[2 * threadIdx.x], c1 = hist[2 * threadIdx.x + 1];
    uint32_t total;
    const uint32_t base = med_block_scan(c0 + c1, s_w, &total);
    if (pass == 0) {
      if (total == 0u) {  // no eligible pixel: no cap
        if (threadIdx.x == 0) cap_out[blockIdx.x] = INFINITY;
        return;
      }
      k = (total - 1u) / 2u;
    }
    if (base <= k && k < base + c0) {
      s_sel[0] = 2u * threadIdx.x;
      s_sel[1] = base;
    } else if (base + c0 <= k && k < base + c0 + c1) {
      s_sel[0] = 2u * threadIdx.x + 1u;
      s_sel[1] = base + c0;
    }
    __syncthreads();
    prefix = (prefix << width[pass]) | s_sel[0];
    k -= s_sel[1];
    __syncthreads();
  }
  if (threadIdx.x == 0) cap_out[blockIdx.x] = factor * __uint_as_float(prefix);
}

void launch_loss_median(const Plan &p, const ViewInfo *views, const float *px_loss, const uint8_t *pmask,
                        float factor, float *cap_out, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_median, dim3((unsigned)p.n_views), dim3(MED_BLOCK), 0, s, views, px_loss, pmask,
                     factor, cap_out);
}

}  // namespace gsr
