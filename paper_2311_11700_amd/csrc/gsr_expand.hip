// Adaptive expansion of the Gaussian map (GS-SLAM Sec. 3.2): the adding
// step (Eq. 8) marks the pixels of rendered keyframes whose cumulative
// opacity is too low or whose rendered depth is too far from the observed
// one and appends a new Gaussian at the back-projection of each (initialised
// as at map initialisation, Eq. 7); the deleting step (Eq. 9) decays the
// opacity of Gaussians floating in front of the observed surface.
//
// Decisions are taken in FP64 on the float32 inputs with contraction off,
// so the masks agree bit for bit with an FP64 reference in the same order.
#pragma clang fp contract(off)

#include <math.h>

#include "gsr_internal.h"

namespace gsr {

// One bit per pixel, one 64-bit word per (chunk, round, wavefront): pixel
// p = chunk * EXPAND_CHUNK + round * BLOCK + thread is bit (thread & 63) of
// word (chunk * EXPAND_ROUNDS + round) * 4 + (thread >> 6) -- so the words of
// a chunk hold its pixels in pixel order.
constexpr int EXPAND_ROUNDS = EXPAND_CHUNK / BLOCK;

struct ExpandArgs {
  const float *T_final, *depth, *depth_obs, *rgb_obs;
  double tau_T, tau_D;
  int64_t total_pixels;
};

// Eq. 8 on one pixel: a reading to back-project and (A < tau_T or
// |D - D_hat| > tau_D), A = 1 - T_final the cumulative opacity.
__device__ __forceinline__ bool unreliable(const ExpandArgs &a, int64_t p) {
  const double T = a.T_final[p], Dh = a.depth[p], D = a.depth_obs[p];
  return D > 0.0 && ((1.0 - T) < a.tau_T || fabs(D - Dh) > a.tau_D);
}

// Pass 1: flags of a chunk of pixels as ballot words, the chunk's count, and
// the optional per-pixel flag bytes.
__global__ __launch_bounds__(BLOCK) void k_expand_flags(ExpandArgs a, unsigned long long *__restrict__ bits,
                                                        uint32_t *__restrict__ cnt, uint8_t *__restrict__ pflag) {
  __shared__ uint32_t s_w[BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t mine = 0u;
  for (int r = 0; r < EXPAND_ROUNDS; ++r) {
    const int64_t p = (int64_t)blockIdx.x * EXPAND_CHUNK + (int64_t)r * BLOCK + threadIdx.x;
    const bool f = p < a.total_pixels && unreliable(a, p);
    const unsigned long long b = __ballot(f);
    if (lane == 0) {
      bits[((size_t)blockIdx.x * EXPAND_ROUNDS + r) * (BLOCK / 64) + wave] = b;
      mine += (uint32_t)__popcll(b);
    }
    if (pflag && p < a.total_pixels) pflag[p] = f ? 1 : 0;
  }
  if (lane == 0) s_w[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

// Pass 2 (one block): exclusive scan of the chunk counts in place; the
// total goes to *count.
__global__ __launch_bounds__(1024) void k_expand_scan(uint32_t *__restrict__ cnt, int n_chunks,
                                                      int64_t *__restrict__ count) {
  __shared__ uint32_t s_w[16];
  __shared__ unsigned long long s_carry;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0ull;
  __syncthreads();
  for (int base = 0; base < n_chunks; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const uint32_t v = i < n_chunks ? cnt[i] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t pre = 0u, tot = 0u;
    for (int w = 0; w < 16; ++w) {
      pre += w < wave ? s_w[w] : 0u;
      tot += s_w[w];
    }
    const unsigned long long carry = s_carry;
    if (i < n_chunks) cnt[i] = (uint32_t)(carry + pre + x - v);
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = (int64_t)s_carry;
}

struct AddOut {
  float *mean, *log_scale, *quat, *opacity_logit, *rgb, *sh;
  int64_t n, capacity;
  float scale_factor, logit_init;
};

// Pass 3: each unreliable pixel's rank in pixel order from the ballot words,
// and its new Gaussian at index n + rank when that fits the capacity.
__global__ __launch_bounds__(BLOCK) void k_expand_write(ExpandArgs a, const unsigned long long *__restrict__ bits,
                                                        const uint32_t *__restrict__ off,
                                                        const gsr_camera *__restrict__ cams,
                                                        const ViewInfo *__restrict__ views, int n_views, AddOut o) {
  __shared__ unsigned long long s_bits[EXPAND_ROUNDS * (BLOCK / 64)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t wbase = (size_t)blockIdx.x * EXPAND_ROUNDS * (BLOCK / 64);
  if (threadIdx.x < EXPAND_ROUNDS * (BLOCK / 64)) s_bits[threadIdx.x] = bits[wbase + threadIdx.x];
  __syncthreads();
  // Words before this thread's first word, in pixel order.
  int64_t rank = off[blockIdx.x];
  for (int r = 0; r < EXPAND_ROUNDS; ++r) {
    const int wi = r * (BLOCK / 64) + wave;
    uint32_t before = 0u;
    for (int w = 0; w < wi; ++w) before += (uint32_t)__popcll(s_bits[w]);
    const unsigned long long b = s_bits[wi];
    if (!((b >> lane) & 1ull)) continue;
    const int64_t p = (int64_t)blockIdx.x * EXPAND_CHUNK + (int64_t)r * BLOCK + threadIdx.x;
    const int64_t k = o.n + rank + before + (uint32_t)__popcll(b & lanemask_lt());
    if (k >= o.capacity) continue;
    // View of pixel p (the views' pixel offsets ascend).
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (views[mid].pix_off <= p) lo = mid; else hi = mid - 1;
    }
    const ViewInfo vi = views[lo];
    const gsr_camera &cam = cams[lo];
    const int64_t q = p - vi.pix_off;
    const double x = (double)(q % vi.W), y = (double)(q / vi.W);
    const double D = a.depth_obs[p];
    const double fx = cam.fx, fy = cam.fy;
    const double xc = D * (x - (double)cam.cx) / fx;
    const double yc = D * (y - (double)cam.cy) / fy;
    const double zc = D;
    const double dx = xc - (double)cam.t[0], dy = yc - (double)cam.t[1], dz = zc - (double)cam.t[2];
    const float *R = cam.R;
    // X = R^T (X_c - t), each component summed in row order.
    const double X0 = ((double)R[0] * dx + (double)R[3] * dy) + (double)R[6] * dz;
    const double X1 = ((double)R[1] * dx + (double)R[4] * dy) + (double)R[7] * dz;
    const double X2 = ((double)R[2] * dx + (double)R[5] * dy) + (double)R[8] * dz;
    const float ls = (float)log((double)o.scale_factor * D / sqrt(fx * fy));
    o.mean[3 * k] = (float)X0;
    o.mean[3 * k + 1] = (float)X1;
    o.mean[3 * k + 2] = (float)X2;
    o.log_scale[3 * k] = ls;
    o.log_scale[3 * k + 1] = ls;
    o.log_scale[3 * k + 2] = ls;
    reinterpret_cast<float4 *>(o.quat)[k] = make_float4(1.f, 0.f, 0.f, 0.f);
    o.opacity_logit[k] = o.logit_init;
    const int64_t HW = (int64_t)vi.W * vi.H;
    const float *c = a.rgb_obs + 3 * vi.pix_off + q;
    const float c0 = c[0], c1 = c[HW], c2 = c[2 * HW];
    if (o.rgb) {
      o.rgb[3 * k] = c0;
      o.rgb[3 * k + 1] = c1;
      o.rgb[3 * k + 2] = c2;
    }
    if (o.sh) {
      // The observed colour in the constant term (Y_0 = SH_C0), none in the
      // linear terms.
      float *sk = o.sh + 12 * k;
      sk[0] = (float)((double)c0 / SH_C0);
      sk[1] = (float)((double)c1 / SH_C0);
      sk[2] = (float)((double)c2 / SH_C0);
#pragma unroll
      for (int j = 3; j < 12; ++j) sk[j] = 0.f;
    }
  }
}

void launch_expand_add(const Plan &p, const ViewInfo *views, const gsr_camera *cams, const float *T_final,
                       const float *depth, const float *depth_obs, const float *rgb_obs, float tau_T, float tau_D,
                       float scale_factor, float logit_init, const Workspace &ws, int64_t n, int64_t capacity,
                       const gsr_gaussians_out &out, uint8_t *pixel_flag, int64_t *count, hipStream_t s) {
  const int n_chunks = (int)((p.total_pixels + EXPAND_CHUNK - 1) / EXPAND_CHUNK);
  ExpandArgs a{T_final, depth, depth_obs, rgb_obs, (double)tau_T, (double)tau_D, p.total_pixels};
  hipLaunchKernelGGL(k_expand_flags, dim3(n_chunks), dim3(BLOCK), 0, s, a, ws.expand_bits, ws.expand_cnt,
                     pixel_flag);
  hipLaunchKernelGGL(k_expand_scan, dim3(1), dim3(1024), 0, s, ws.expand_cnt, n_chunks, count);
  AddOut o{out.mean, out.log_scale, out.quat, out.opacity_logit, out.rgb, out.sh, n, capacity, scale_factor,
           logit_init};
  hipLaunchKernelGGL(k_expand_write, dim3(n_chunks), dim3(BLOCK), 0, s, a, ws.expand_bits, ws.expand_cnt, cams,
                     views, p.n_views, o);
}

// Deleting step (Eq. 9): a visible Gaussian whose ray meets the observed
// surface more than gamma beyond it has its opacity scaled by eta.
__global__ __launch_bounds__(BLOCK) void k_expand_delete(gsr_gaussians g, const gsr_camera *__restrict__ cam,
                                                         const float *__restrict__ depth_obs, int W, int H,
                                                         double gamma, double eta, double z_near,
                                                         float *logit_out, uint8_t *__restrict__ decayed) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.n) return;
  const float lam = g.opacity_logit[i];
  bool hit = false;
  if (!g.mask || g.mask[i] != 0) {
    const double mx = g.mean[3 * i], my = g.mean[3 * i + 1], mz = g.mean[3 * i + 2];
    const float *R = cam->R;
    const double x = (((double)R[0] * mx + (double)R[1] * my) + (double)R[2] * mz) + (double)cam->t[0];
    const double y = (((double)R[3] * mx + (double)R[4] * my) + (double)R[5] * mz) + (double)cam->t[1];
    const double z = (((double)R[6] * mx + (double)R[7] * my) + (double)R[8] * mz) + (double)cam->t[2];
    if (z > z_near) {
      const double u = ((double)cam->fx * x) / z + (double)cam->cx;
      const double v = ((double)cam->fy * y) / z + (double)cam->cy;
      const double pxd = floor(u + 0.5), pyd = floor(v + 0.5);
      if (pxd >= 0.0 && pxd < (double)W && pyd >= 0.0 && pyd < (double)H) {
        const double D = depth_obs[(int64_t)pyd * W + (int64_t)pxd];
        // The observed surface point of the pixel lies on the same ray at
        // D / z times X_c: its signed distance beyond the Gaussian.
        if (D > 0.0) hit = (D - z) * sqrt((x * x + y * y) + z * z) / z > gamma;
      }
    }
  }
  float out = lam;
  if (hit) {
    const double o = 1.0 / (1.0 + exp(-(double)lam));
    const double o2 = eta * o;
    out = (float)log(o2 / (1.0 - o2));
  }
  logit_out[i] = out;
  if (decayed) decayed[i] = hit ? 1 : 0;
}

void launch_expand_delete(const gsr_gaussians &g, const gsr_camera *cam, const float *depth_obs, int W, int H,
                          float gamma, float eta, float z_near, float *logit_out, uint8_t *decayed, hipStream_t s) {
  if (g.n > 0)
    hipLaunchKernelGGL(k_expand_delete, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g, cam,
                       depth_obs, W, H, (double)gamma, (double)eta, (double)z_near, logit_out, decayed);
}

}  // namespace gsr
