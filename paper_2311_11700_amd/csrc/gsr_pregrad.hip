// Chain rule from the per-view 2D gradients back to the Gaussian parameters
// and the camera pose (GS-SLAM Eq. 2-3, Eq. 11 and supplement Sec. A).
#include <math.h>

#include "gsr_internal.h"

namespace gsr {

struct PreConstsB {
  float z_near, lowpass, cutoff;
  uint32_t flags;
  float fov_guard;
};

// dst += v, or dst = v when the gradients are overwritten.
__device__ __forceinline__ void put(float &dst, double v, bool overwrite) {
  dst = overwrite ? (float)v : dst + (float)v;
}

// The chain runs in FP64: gfx950 executes FP64 vector arithmetic at the
// non-packed FP32 rate, and near-camera Gaussians put 1/z^3 factors and
// cancelling terms into this chain.
using R = double;

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Rotation matrix of a unit quaternion (w, x, y, z) (supplement eq. q2R).
__device__ __forceinline__ void quat_rot_r(R w, R x, R y, R z, R M[9]) {
  M[0] = R(1) - R(2) * (y * y + z * z);
  M[1] = R(2) * (x * y - w * z);
  M[2] = R(2) * (x * z + w * y);
  M[3] = R(2) * (x * y + w * z);
  M[4] = R(1) - R(2) * (x * x + z * z);
  M[5] = R(2) * (y * z - w * x);
  M[6] = R(2) * (x * z - w * y);
  M[7] = R(2) * (y * z + w * x);
  M[8] = R(1) - R(2) * (x * x + y * y);
}

// ----------------------------------------------------------------------------
// Backward: per Gaussian, loop over the views, chain the per-view 2D
// gradients (u, v, conic, opacity, colour, depth) through Eq. 3 to the
// camera-frame point and covariance, accumulate dL/dmean and dL/dSigma over
// views, then chain dL/dSigma through Eq. 2 to the log-scales and the
// quaternion once.  The pose gradient of each view is the left-perturbation
// derivative rho = sum gX, phi = sum (X_c x gX + 2 vee(G_c Sigma_c - Sigma_c G_c)),
// reduced per block into fixed slots (deterministic order).

// SH: the colour is degree-1 spherical harmonics (instantiated separately so
// that the RGB path carries none of their registers).
// Registers held to two wavefronts per SIMD: the SH instance would otherwise
// take 256 and run one wavefront per SIMD.
template <bool SH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_preprocess_bwd(gsr_gaussians g,
                                                          const gsr_camera *__restrict__ cams,
                                                          int n_views, PreConstsB pc, Workspace ws,
                                                          gsr_grads gr) {
  extern __shared__ double s_dyn[];  // [4 waves][n_views][6]
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool active = i < g.n;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool want_pose = (pc.flags & GSR_POSE_GRAD) && gr.d_pose;
  const bool want_gauss = (pc.flags & GSR_GAUSS_GRAD) != 0;
  const bool approx = (pc.flags & GSR_PAPER_POSE_APPROX) != 0;

  if (want_pose) {
    for (int k = threadIdx.x; k < 4 * n_views * 6; k += BLOCK) s_dyn[k] = 0.;
    __syncthreads();
  }

  R mx = 0, my = 0, mz = 0, qw = 1, qx = 0, qy = 0, qz = 0, qn = 1, s0 = 1, s1 = 1, s2 = 1;
  R opl = 0;
  // Spherical-harmonic coefficients [4][3] (when the colour is view-dependent).
  constexpr bool sh_mode = SH;
  // The linear coefficients as stored (float32, widened where used); the
  // constant term does not enter the direction gradient.
  float shc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) shc[k] = 0.f;
  if (active && sh_mode) {
#pragma unroll
    for (int k = 0; k < 9; ++k) shc[k] = g.sh[12 * i + 3 + k];
  }
  // Gradients of the linear coefficients; the constant term's is Y_0 times
  // the colour gradient summed over the views (gc0..gc2).
  R gsh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) gsh[k] = 0.;
  if (active) {
    mx = g.mean[3 * i]; my = g.mean[3 * i + 1]; mz = g.mean[3 * i + 2];
    s0 = exp((R)g.log_scale[3 * i]); s1 = exp((R)g.log_scale[3 * i + 1]);
    s2 = exp((R)g.log_scale[3 * i + 2]);
    const float4 fq = reinterpret_cast<const float4 *>(g.quat)[i];
    const R q0 = fq.x, q1 = fq.y, q2 = fq.z, q3 = fq.w;
    qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const R inv = qn > 0 ? R(1) / qn : R(0);
    qw = q0 * inv; qx = q1 * inv; qy = q2 * inv; qz = q3 * inv;
    opl = g.opacity_logit[i];
  }
  R Rq[9];
  quat_rot_r(qw, qx, qy, qz, Rq);
  const R v0 = s0 * s0, v1 = s1 * s1, v2 = s2 * s2;
  R S[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[3 * r + c] = Rq[3 * r] * v0 * Rq[3 * c] + Rq[3 * r + 1] * v1 * Rq[3 * c + 1] +
                     Rq[3 * r + 2] * v2 * Rq[3 * c + 2];

  R gm[3] = {0, 0, 0};
  R GS[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  R gop = 0., gc0 = 0., gc1 = 0., gc2 = 0.;

  for (int view = 0; view < n_views; ++view) {
    const int64_t rec = (int64_t)view * g.n + i;
    R g2[NGRAD2D];
    bool has = false;
    if (active && ws.count[rec] != 0u) {
      const double *src = ws.grad2d + rec * NGRAD2D;
#pragma unroll
      for (int k = 0; k < NGRAD2D; ++k) {
        g2[k] = src[k];
        has = has || (g2[k] != 0.);
      }
    }
    R pr[6] = {0, 0, 0, 0, 0, 0};
    if (has) {
      const gsr_camera &cam = cams[view];
      R W[9];
      for (int k = 0; k < 9; ++k) W[k] = cam.R[k];
      const R x = W[0] * mx + W[1] * my + W[2] * mz + (R)cam.t[0];
      const R y = W[3] * mx + W[4] * my + W[5] * mz + (R)cam.t[1];
      const R z = W[6] * mx + W[7] * my + W[8] * mz + (R)cam.t[2];
      R Mt[9], Sc[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Mt[3 * r + c] = W[3 * r] * S[c] + W[3 * r + 1] * S[3 + c] + W[3 * r + 2] * S[6 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Sc[3 * r + c] = Mt[3 * r] * W[3 * c] + Mt[3 * r + 1] * W[3 * c + 1] + Mt[3 * r + 2] * W[3 * c + 2];
      const R fx = cam.fx, fy = cam.fy;
      const R iz = R(1) / z, iz2 = iz * iz, iz3 = iz2 * iz;
      // x/z, y/z as they enter J (limited by the guard); a limited ratio no
      // longer depends on x (or y), and J then depends on z through 1/z only.
      R rxz = x * iz, ryz = y * iz;
      R free_x = 1., free_y = 1.;
      if (pc.fov_guard > 0.f) {
        const R lx = (R)pc.fov_guard * (0.5 * (R)cam.width) / fx;
        const R ly = (R)pc.fov_guard * (0.5 * (R)cam.height) / fy;
        if (rxz > lx || rxz < -lx) { rxz = rxz > 0. ? lx : -lx; free_x = 0.; }
        if (ryz > ly || ryz < -ly) { ryz = ryz > 0. ? ly : -ly; free_y = 0.; }
      }
      const R J00 = fx * iz, J02 = -fx * rxz * iz, J11 = fy * iz, J12 = -fy * ryz * iz;
      // J Sigma_c (2x3)
      R JS0[3], JS1[3];
      for (int c = 0; c < 3; ++c) {
        JS0[c] = J00 * Sc[c] + J02 * Sc[6 + c];
        JS1[c] = J11 * Sc[3 + c] + J12 * Sc[6 + c];
      }
      const R A = JS0[0] * J00 + JS0[2] * J02 + pc.lowpass;
      const R B = JS0[1] * J11 + JS0[2] * J12;
      const R C = JS1[1] * J11 + JS1[2] * J12 + pc.lowpass;
      const R idet = 1. / (A * C - B * B);
      const R ca = C * idet, cb = -B * idet, cc = A * idet;
      // dL/dSigma' = -M G_M M with M the conic, G_M = [[ga, gb/2], [gb/2, gc]].
      const R n00 = g2[2], n01 = 0.5 * g2[3], n11 = g2[4];
      const R P00 = ca * n00 + cb * n01, P01 = ca * n01 + cb * n11;
      const R P10 = cb * n00 + cc * n01, P11 = cb * n01 + cc * n11;
      const R G00 = -(P00 * ca + P01 * cb), G01 = -(P00 * cb + P01 * cc),
                  G11 = -(P10 * cb + P11 * cc);
      // dL/dSigma_c = J^T G J (symmetric 3x3).
      R GSc[9];
      GSc[0] = J00 * J00 * G00;
      GSc[1] = J00 * J11 * G01;
      GSc[2] = J00 * (G00 * J02 + G01 * J12);
      GSc[4] = J11 * J11 * G11;
      GSc[5] = J11 * (G01 * J02 + G11 * J12);
      GSc[8] = J02 * J02 * G00 + 2. * J02 * J12 * G01 + J12 * J12 * G11;
      GSc[3] = GSc[1]; GSc[6] = GSc[2]; GSc[7] = GSc[5];
      // dL/dJ = 2 G J Sigma_c (only the entries J depends on are needed).
      const R GJ00 = 2. * (G00 * JS0[0] + G01 * JS1[0]);
      const R GJ02 = 2. * (G00 * JS0[2] + G01 * JS1[2]);
      const R GJ11 = 2. * (G01 * JS0[1] + G11 * JS1[1]);
      const R GJ12 = 2. * (G01 * JS0[2] + G11 * JS1[2]);
      const R gu = g2[0], gv = g2[1], gzd = g2[9];
      // Through the projected centre and depth.
      const R pX0 = gu * fx * iz;
      const R pX1 = gv * fy * iz;
      const R pX2 = -gu * fx * x * iz2 - gv * fy * y * iz2 + gzd;
      // Through J (part of the Sigma' path): J02 = -fx r/z with r = x/z (or
      // its limit), dJ02/dx = -fx/z^2 while r is free, dJ02/dz = fx r/z^2
      // (+ fx x/z^3 while r is free); J12 likewise.
      const R jX0 = -GJ02 * fx * iz2 * free_x;
      const R jX1 = -GJ12 * fy * iz2 * free_y;
      const R jX2 = -GJ00 * fx * iz2 + GJ02 * fx * (rxz * iz2 + free_x * x * iz3) - GJ11 * fy * iz2 +
                        GJ12 * fy * (ryz * iz2 + free_y * y * iz3);
      const R gX0 = pX0 + jX0, gX1 = pX1 + jX1, gX2 = pX2 + jX2;
      if (want_gauss) {
        gm[0] += W[0] * gX0 + W[3] * gX1 + W[6] * gX2;
        gm[1] += W[1] * gX0 + W[4] * gX1 + W[7] * gX2;
        gm[2] += W[2] * gX0 + W[5] * gX1 + W[8] * gX2;
        // W^T GSc W
        R T9[9];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c)
            T9[3 * r + c] = W[r] * GSc[c] + W[3 + r] * GSc[3 + c] + W[6 + r] * GSc[6 + c];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c)
            GS[3 * r + c] += T9[3 * r] * W[c] + T9[3 * r + 1] * W[3 + c] + T9[3 * r + 2] * W[6 + c];
        gop += g2[5];
        gc0 += g2[6]; gc1 += g2[7]; gc2 += g2[8];
      }
      // Spherical-harmonic colour: coefficient gradient Y (x) dL/dc and, through
      // the viewing direction d = v / |v| (v = mean - o, o = -W^T t),
      // dL/dv = (I - d d^T) dL/dd / |v|, which adds to the mean and, since a
      // left perturbation moves o by -W^T rho, W dL/dv to the pose's rho.
      R gv0 = 0., gv1 = 0., gv2 = 0.;
      if (sh_mode) {
        const R t0 = cam.t[0], t1 = cam.t[1], t2 = cam.t[2];
        const R vx = mx + (W[0] * t0 + W[3] * t1 + W[6] * t2);
        const R vy = my + (W[1] * t0 + W[4] * t1 + W[7] * t2);
        const R vz = mz + (W[2] * t0 + W[5] * t1 + W[8] * t2);
        const R il = R(1) / sqrt(vx * vx + vy * vy + vz * vz);
        const R dx = vx * il, dy = vy * il, dz = vz * il;
        const R Y[3] = {SH_C1 * dy, SH_C1 * dz, SH_C1 * dx};
        const R gc[3] = {g2[6], g2[7], g2[8]};
        if (want_gauss) {
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gsh[3 * k + ch] += Y[k] * gc[ch];
        }
        R gY1 = 0., gY2 = 0., gY3 = 0.;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          gY1 += (R)shc[ch] * gc[ch];
          gY2 += (R)shc[3 + ch] * gc[ch];
          gY3 += (R)shc[6 + ch] * gc[ch];
        }
        const R gdx = SH_C1 * gY3, gdy = SH_C1 * gY1, gdz = SH_C1 * gY2;
        const R dot = dx * gdx + dy * gdy + dz * gdz;
        gv0 = (gdx - dx * dot) * il;
        gv1 = (gdy - dy * dot) * il;
        gv2 = (gdz - dz * dot) * il;
        if (want_gauss) {
          gm[0] += gv0;
          gm[1] += gv1;
          gm[2] += gv2;
        }
      }
      if (want_pose) {
        const R rX0 = approx ? pX0 : gX0, rX1 = approx ? pX1 : gX1, rX2 = approx ? pX2 : gX2;
        pr[0] = rX0; pr[1] = rX1; pr[2] = rX2;
        pr[3] = y * rX2 - z * rX1;
        pr[4] = z * rX0 - x * rX2;
        pr[5] = x * rX1 - y * rX0;
        if (!approx) {
          // B = Sigma_c GSc; phi += 2 (B12 - B21, B20 - B02, B01 - B10).
          R Bm[9];
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
              Bm[3 * r + c] = Sc[3 * r] * GSc[c] + Sc[3 * r + 1] * GSc[3 + c] + Sc[3 * r + 2] * GSc[6 + c];
          pr[3] += 2. * (Bm[5] - Bm[7]);
          pr[4] += 2. * (Bm[6] - Bm[2]);
          pr[5] += 2. * (Bm[1] - Bm[3]);
        }
        if (sh_mode) {
          pr[0] += W[0] * gv0 + W[1] * gv1 + W[2] * gv2;
          pr[1] += W[3] * gv0 + W[4] * gv1 + W[5] * gv2;
          pr[2] += W[6] * gv0 + W[7] * gv1 + W[8] * gv2;
        }
      }
    }
    if (want_pose && __any(has)) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const R t = wave_sum_d(pr[k]);
        if (lane == 0) s_dyn[(wave * n_views + view) * 6 + k] = t;
      }
    }
  }

  if (active && want_gauss) {
    // Eq. 2 backward: Sigma = Rq diag(s^2) Rq^T.
    R GR[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const R vv = c == 0 ? v0 : (c == 1 ? v1 : v2);
        GR[3 * r + c] = 2. * (GS[3 * r] * Rq[c] + GS[3 * r + 1] * Rq[3 + c] + GS[3 * r + 2] * Rq[6 + c]) * vv;
      }
    R d[3];
    for (int k = 0; k < 3; ++k) {
      R acc = 0.;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) acc += Rq[3 * r + k] * GS[3 * r + c] * Rq[3 * c + k];
      d[k] = acc;
    }
    const R gl0 = 2. * v0 * d[0], gl1 = 2. * v1 * d[1], gl2 = 2. * v2 * d[2];
    const R w = qw, x = qx, y = qy, z = qz;
    const R gw = 2. * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    const R gx = 2. * (y * GR[1] + z * GR[2] + y * GR[3] - 2. * x * GR[4] - w * GR[5] + z * GR[6] +
                            w * GR[7] - 2. * x * GR[8]);
    const R gy = 2. * (-2. * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] +
                            z * GR[7] - 2. * y * GR[8]);
    const R gz = 2. * (-2. * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2. * z * GR[4] + y * GR[5] +
                            x * GR[6] + y * GR[7]);
    const R dotq = w * gw + x * gx + y * gy + z * gz;
    const R iq = qn > 0. ? 1. / qn : 0.;
    const R o = R(1) / (R(1) + exp(-opl));
    const bool ow = (pc.flags & GSR_GRAD_OVERWRITE) != 0;
    if (gr.d_mean) {
      put(gr.d_mean[3 * i], gm[0], ow);
      put(gr.d_mean[3 * i + 1], gm[1], ow);
      put(gr.d_mean[3 * i + 2], gm[2], ow);
    }
    if (gr.d_log_scale) {
      put(gr.d_log_scale[3 * i], gl0, ow);
      put(gr.d_log_scale[3 * i + 1], gl1, ow);
      put(gr.d_log_scale[3 * i + 2], gl2, ow);
    }
    if (gr.d_quat) {
      float4 *dq = reinterpret_cast<float4 *>(gr.d_quat) + i;
      float4 cur = ow ? make_float4(0.f, 0.f, 0.f, 0.f) : *dq;
      cur.x += (float)((gw - w * dotq) * iq);
      cur.y += (float)((gx - x * dotq) * iq);
      cur.z += (float)((gy - y * dotq) * iq);
      cur.w += (float)((gz - z * dotq) * iq);
      *dq = cur;
    }
    if (gr.d_opacity_logit) put(gr.d_opacity_logit[i], gop * o * (R(1) - o), ow);
    if (sh_mode && gr.d_sh) {
      put(gr.d_sh[12 * i], SH_C0 * gc0, ow);
      put(gr.d_sh[12 * i + 1], SH_C0 * gc1, ow);
      put(gr.d_sh[12 * i + 2], SH_C0 * gc2, ow);
#pragma unroll
      for (int k = 0; k < 9; ++k) put(gr.d_sh[12 * i + 3 + k], gsh[k], ow);
    }
    if (gr.d_rgb && !sh_mode) {
      put(gr.d_rgb[3 * i], gc0, ow);
      put(gr.d_rgb[3 * i + 1], gc1, ow);
      put(gr.d_rgb[3 * i + 2], gc2, ow);
    }
  }

  if (want_pose) {
    __syncthreads();
    const int V6 = n_views * 6;
    R *dst = ws.pose_part + (int64_t)blockIdx.x * V6;
    for (int k = threadIdx.x; k < V6; k += BLOCK)
      dst[k] = s_dyn[k] + s_dyn[V6 + k] + s_dyn[2 * V6 + k] + s_dyn[3 * V6 + k];
  }
}

// Deterministic reduction of the per-block pose partials: one block per
// (view, component), fixed summation order.
__global__ __launch_bounds__(BLOCK) void k_pose_reduce(const double *__restrict__ part, int n_blocks,
                                                       int n_views, int overwrite, float *__restrict__ d_pose) {
  __shared__ double red[BLOCK];
  const int vc = blockIdx.x;  // view * 6 + component
  double acc = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += BLOCK) acc += part[(int64_t)b * n_views * 6 + vc];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) put(d_pose[vc], red[0], overwrite != 0);
}

void launch_preprocess_backward(const Plan &p, const gsr_gaussians &g, const gsr_camera *cams,
                                const gsr_config &cfg, const Workspace &ws, const gsr_grads &gr,
                                hipStream_t s) {
  const bool want_pose = (cfg.flags & GSR_POSE_GRAD) && gr.d_pose;
  if (g.n == 0) {
    // No Gaussian, no gradient: an overwritten pose gradient is zero.
    if (want_pose && (cfg.flags & GSR_GRAD_OVERWRITE)) launch_fill_f32(gr.d_pose, 0.f, (int64_t)p.n_views * 6, s);
    return;
  }
  PreConstsB pc{cfg.z_near, cfg.lowpass, cfg.cutoff_sigma, cfg.flags, cfg.fov_guard};
  const size_t lds = want_pose ? (size_t)4 * p.n_views * 6 * sizeof(double) : 0;
  hipLaunchKernelGGL(g.sh ? k_preprocess_bwd<true> : k_preprocess_bwd<false>, dim3(p.n_pose_blocks), dim3(BLOCK), lds, s, g, cams,
                     p.n_views, pc, ws, gr);
  if (want_pose)
    hipLaunchKernelGGL(k_pose_reduce, dim3(p.n_views * 6), dim3(BLOCK), 0, s, ws.pose_part, p.n_pose_blocks,
                       p.n_views, (cfg.flags & GSR_GRAD_OVERWRITE) ? 1 : 0, gr.d_pose);
}

}  // namespace gsr
