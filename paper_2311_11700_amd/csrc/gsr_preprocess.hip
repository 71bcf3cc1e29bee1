// Per-(view, Gaussian) projection: camera-frame centre, EWA screen-space
// covariance and its conic, opacity, tile rectangle and depth sort key
// (GS-SLAM Eq. 2-3, supplement eq. q2R).
//
// Forward geometry runs in FP64: gfx950 executes FP64 vector arithmetic at
// the FP32 non-packed rate, and computing the binning quantities (depth sort
// key, tile rectangle) in FP64 with contraction disabled makes them agree bit
// for bit with an FP64 reference evaluated in the same order.  The values the
// rasteriser consumes are rounded to FP32 once, at the end.
#pragma clang fp contract(off)

#include <math.h>

#include "gsr_internal.h"

namespace gsr {

struct PreConsts {
  float z_near, lowpass, cutoff;
  uint32_t flags;
  float fov_guard;
  float alpha_min;
  int clear_grad2d;  // zero each record's grad2d row (start of a fused step)
  float *loss_zero;  // zeroed by one thread when not null
  int order_total;   // > 0: block 0 writes the rasteriser's work order of this many tiles
};

// Rotation matrix of a unit quaternion (w, x, y, z) (GS-SLAM supplement,
// eq. q2R), row-major.
template <typename T>
__device__ __forceinline__ void quat_rot(T w, T x, T y, T z, T R[9]) {
  R[0] = T(1) - T(2) * (y * y + z * z);
  R[1] = T(2) * (x * y - w * z);
  R[2] = T(2) * (x * z + w * y);
  R[3] = T(2) * (x * y + w * z);
  R[4] = T(1) - T(2) * (x * x + z * z);
  R[5] = T(2) * (y * z - w * x);
  R[6] = T(2) * (x * z - w * y);
  R[7] = T(2) * (y * z + w * x);
  R[8] = T(1) - T(2) * (x * x + y * y);
}

// Project record rec = view * n + i; returns its depth sort key (float32
// depth bits, 0xFFFFFFFF when culled).  SH: spherical-harmonic colour.
template <bool SH>
__device__ __forceinline__ uint32_t project_record(const gsr_gaussians &g, const gsr_camera *__restrict__ cams,
                                                   const ViewInfo *__restrict__ views, const PreConsts &pc,
                                                   const Workspace &ws, int view, int64_t i, int64_t rec) {
  const ViewInfo vi = views[view];
  const gsr_camera &cam = cams[view];

  const float fm0 = g.mean[3 * i], fm1 = g.mean[3 * i + 1], fm2 = g.mean[3 * i + 2];
  const float fl0 = g.log_scale[3 * i], fl1 = g.log_scale[3 * i + 1], fl2 = g.log_scale[3 * i + 2];
  const float4 fq = reinterpret_cast<const float4 *>(g.quat)[i];
  const float fop = g.opacity_logit[i];
  // Colour: RGB, or the 12 spherical-harmonic coefficients [4][3].
  constexpr int ncol = SH ? 12 : 3;
  float col[ncol];
  const float *csrc = SH ? g.sh + 12 * i : g.rgb + 3 * i;
  bool colour_ok = true;
#pragma unroll
  for (int k = 0; k < ncol; ++k) {
    col[k] = csrc[k];
    colour_ok = colour_ok && isfinite(col[k]);
  }

  bool ok = isfinite(fm0) && isfinite(fm1) && isfinite(fm2) && isfinite(fl0) && isfinite(fl1) &&
            isfinite(fl2) && isfinite(fq.x) && isfinite(fq.y) && isfinite(fq.z) && isfinite(fq.w) &&
            isfinite(fop) && colour_ok;
  if (g.mask) ok = ok && g.mask[i] != 0;

  // Camera-frame centre, each row summed left to right (this is the exact
  // sequence behind the float32 depth key).
  const double mx = fm0, my = fm1, mz = fm2;
  const double W0 = cam.R[0], W1 = cam.R[1], W2 = cam.R[2], W3 = cam.R[3], W4 = cam.R[4],
               W5 = cam.R[5], W6 = cam.R[6], W7 = cam.R[7], W8 = cam.R[8];
  const double x = ((W0 * mx + W1 * my) + W2 * mz) + (double)cam.t[0];
  const double y = ((W3 * mx + W4 * my) + W5 * mz) + (double)cam.t[1];
  const double z = ((W6 * mx + W7 * my) + W8 * mz) + (double)cam.t[2];
  ok = ok && (z > (double)pc.z_near);

  // Covariance (Eq. 2).
  double qw = fq.x, qx = fq.y, qy = fq.z, qz = fq.w;
  const double qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  ok = ok && (qn > 0.0);
  double Rq[9];
  {
    const double inv = ok ? qn : 1.0;
    qw /= inv; qx /= inv; qy /= inv; qz /= inv;
    quat_rot<double>(qw, qx, qy, qz, Rq);
  }
  const double s0 = exp((double)fl0), s1 = exp((double)fl1), s2 = exp((double)fl2);
  const double q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
  double S[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[3 * r + c] = (Rq[3 * r] * q0 * Rq[3 * c] + Rq[3 * r + 1] * q1 * Rq[3 * c + 1]) +
                     Rq[3 * r + 2] * q2 * Rq[3 * c + 2];
  // Camera-frame covariance W S W^T.
  const double Wm[9] = {W0, W1, W2, W3, W4, W5, W6, W7, W8};
  double M[9], Sc[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      M[3 * r + c] = (Wm[3 * r] * S[c] + Wm[3 * r + 1] * S[3 + c]) + Wm[3 * r + 2] * S[6 + c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      Sc[3 * r + c] = (M[3 * r] * Wm[3 * c] + M[3 * r + 1] * Wm[3 * c + 1]) + M[3 * r + 2] * Wm[3 * c + 2];
  // EWA projection (Eq. 3): J = [[fx/z, 0, -fx (x/z)/z], [0, fy/z, -fy (y/z)/z]],
  // with x/z and y/z limited to +-g W/(2 fx), +-g H/(2 fy) when the guard g
  // is on (the projected centre below is not limited).
  const double fx = cam.fx, fy = cam.fy;
  const double zz = ok ? z : 1.0;
  double rx_ = x / zz, ry_ = y / zz;
  if (pc.fov_guard > 0.f) {
    const double lx = (double)pc.fov_guard * (0.5 * (double)vi.W) / fx;
    const double ly = (double)pc.fov_guard * (0.5 * (double)vi.H) / fy;
    rx_ = fmin(lx, fmax(-lx, rx_));
    ry_ = fmin(ly, fmax(-ly, ry_));
  }
  const double J00 = fx / zz, J02 = -(fx * rx_) / zz;
  const double J11 = fy / zz, J12 = -(fy * ry_) / zz;
  const double T00 = J00 * Sc[0] + J02 * Sc[6], T01 = J00 * Sc[1] + J02 * Sc[7],
               T02 = J00 * Sc[2] + J02 * Sc[8];
  const double T11 = J11 * Sc[4] + J12 * Sc[7], T12 = J11 * Sc[5] + J12 * Sc[8];
  const double A = (T00 * J00 + T02 * J02) + (double)pc.lowpass;
  const double B = T01 * J11 + T02 * J12;
  const double C = (T11 * J11 + T12 * J12) + (double)pc.lowpass;
  const double det = A * C - B * B;
  ok = ok && (det > 0.0);

  const double u = (fx * x) / zz + (double)cam.cx;
  const double v = (fy * y) / zz + (double)cam.cy;

  int tx0 = 0, tx1 = vi.TX - 1, ty0 = 0, ty1 = vi.TY - 1;
  if (!(pc.flags & GSR_FULL_RECT) && ok) {
    const double rx = (double)pc.cutoff * sqrt(A), ry = (double)pc.cutoff * sqrt(C);
    const double bx0 = floor((u - rx) / (double)TILE), bx1 = floor((u + rx) / (double)TILE);
    const double by0 = floor((v - ry) / (double)TILE), by1 = floor((v + ry) / (double)TILE);
    const double cx0 = fmax(0.0, bx0), cx1 = fmin((double)(vi.TX - 1), bx1);
    const double cy0 = fmax(0.0, by0), cy1 = fmin((double)(vi.TY - 1), by1);
    ok = ok && (cx0 <= cx1) && (cy0 <= cy1);
    if (ok) {
      tx0 = (int)cx0; tx1 = (int)cx1; ty0 = (int)cy0; ty1 = (int)cy1;
    }
  }

  if (!ok) {
    ws.count[rec] = 0u;
    return 0xFFFFFFFFu;
  }
  // Only records that enter tile lists receive or give back 2D gradients.
  if (pc.clear_grad2d) {
    double2 *gz = reinterpret_cast<double2 *>(ws.grad2d + rec * NGRAD2D);
#pragma unroll
    for (int k = 0; k < NGRAD2D / 2; ++k) gz[k] = make_double2(0.0, 0.0);
  }
  const float zf = (float)z;
  const float uh = (float)u, vh = (float)v;
  const float op = (float)(1.0 / (1.0 + exp(-(double)fop)));
  const float4 fa = make_float4(uh, (float)(u - (double)uh), vh, (float)(v - (double)vh));
  const float4 fb = make_float4((float)(C / det), (float)(-B / det), (float)(A / det), op);
  ws.recA[rec] = fa;
  ws.recB[rec] = fb;
  float fc0 = col[0], fc1 = col[1], fc2 = col[2];
  if constexpr (SH) {
    // Degree-1 spherical harmonics of the viewing direction d from the
    // camera centre -W^T t to the mean: Y_0 = 1/(2 sqrt(pi)),
    // (Y_1, Y_2, Y_3) = sqrt(3/(4 pi)) (d_y, d_z, d_x).
    const double t0 = cam.t[0], t1 = cam.t[1], t2 = cam.t[2];
    const double vx = mx + ((W0 * t0 + W3 * t1) + W6 * t2);
    const double vy = my + ((W1 * t0 + W4 * t1) + W7 * t2);
    const double vz = mz + ((W2 * t0 + W5 * t1) + W8 * t2);
    const double il = 1.0 / sqrt((vx * vx + vy * vy) + vz * vz);
    const double Y0 = SH_C0, Y1 = SH_C1 * (vy * il), Y2 = SH_C1 * (vz * il), Y3 = SH_C1 * (vx * il);
    double c[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      c[ch] = ((Y0 * (double)col[ch] + Y1 * (double)col[3 + ch]) + Y2 * (double)col[6 + ch]) + Y3 * (double)col[9 + ch];
    fc0 = (float)c[0];
    fc1 = (float)c[1];
    fc2 = (float)c[2];
  }
  ws.recC[rec] = make_float4(fc0, fc1, fc2, zf);
  // Every tile of the rectangle gets a pair; the emission marks the ones the
  // alpha support does not reach (none in the full-rectangle mode or
  // without an alpha threshold).
  const bool cull = !(pc.flags & GSR_FULL_RECT) && pc.alpha_min > 0.f;
  if (cull) {
    Support sp;
    if (!support_of(fa, fb, pc.alpha_min, sp)) {
      sp.U = sp.V = sp.t = sp.dys = sp.ra = 0.0;
      sp.hy = -1.0;  // no row reaches it: every pair is dropped
    }
    ws.support[rec] = sp;
  }
  ws.tinfo[rec] = make_uint4((uint32_t)vi.tile_off, (uint32_t)vi.TX | (cull ? 0x80000000u : 0u),
                             (uint32_t)tx0 | ((uint32_t)tx1 << 16), (uint32_t)ty0 | ((uint32_t)ty1 << 16));
  ws.count[rec] = (uint32_t)(tx1 - tx0 + 1) * (uint32_t)(ty1 - ty0 + 1);
  return __float_as_uint(zf);
}

// One block per sort tile of the depth sort: project its records, write the
// depth keys and record ids of the visible ones to the front of the tile's
// slots in record order (the depth sort reads only those, so culled records
// never enter the sort), and count the keys' first radix digit (bits 0-7)
// for the sort's first pass.  Block 0 also resets the per-call header words
// (and the fused step's loss when it is overwritten).
constexpr int PRE_BLOCK = BLOCK * SORT_ITEMS_DEPTH;
template <bool SH>
__global__ __launch_bounds__(PRE_BLOCK) void k_preprocess(gsr_gaussians g, const gsr_camera *__restrict__ cams,
                                                          const ViewInfo *__restrict__ views, PreConsts pc,
                                                          Workspace ws, int n_views, int max_tiles) {
  constexpr int NW = PRE_BLOCK / 64;
  __shared__ uint32_t cnt[RADIX];
  __shared__ uint32_t s_wv[NW];
  __shared__ uint32_t s_qcnt[RADIX], s_qcur[RADIX], s_qw[NW], s_timed;
  const int64_t rec = (int64_t)blockIdx.x * PRE_BLOCK + threadIdx.x;
  const int wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    reset_header_words(ws.hdr);
    s_timed = ws.hdr[HDR_COSTS];  // read by the thread that reset the header
    if (pc.loss_zero) *pc.loss_zero = 0.f;
  }
  if (blockIdx.x == 0 && pc.order_total > 0) {
    // The rasteriser's work order for this step, from the tile durations
    // the last fused step recorded (the other blocks cover its time).
    __syncthreads();
    order_tiles<PRE_BLOCK>(ws.tile_cost, s_timed != 0u, pc.order_total, ws.queue, s_qcnt, s_qcur, s_qw);
  }
  if (threadIdx.x < RADIX) cnt[threadIdx.x] = 0u;
  uint32_t key = 0xFFFFFFFFu;
  if (rec < g.n * (int64_t)n_views) {
    const int view = (int)(rec / g.n);
    key = project_record<SH>(g, cams, views, pc, ws, view, rec - (int64_t)view * g.n, rec);
  }
  // Culled records have the key 0xFFFFFFFF (a visible depth is a positive
  // finite float, whose bits are below it).
  const bool vis = key != 0xFFFFFFFFu;
  const uint64_t vmask = __ballot(vis);
  if ((threadIdx.x & 63) == 0) s_wv[wave] = (uint32_t)__popcll(vmask);
  __syncthreads();
  uint32_t before = 0u, total = 0u;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    before += w < wave ? s_wv[w] : 0u;
    total += s_wv[w];
  }
  if (vis) {
    const int64_t pos = (int64_t)blockIdx.x * PRE_BLOCK + before + (uint32_t)__popcll(vmask & lanemask_lt());
    ws.dkeys[0][pos] = key;
    ws.dvals[0][pos] = (uint32_t)rec;
  }
  const uint32_t d = key & (RADIX - 1u);
  const uint64_t peers = match_digit(d, RADIX_BITS, vmask);
  if (vis && (peers & lanemask_lt()) == 0ull) atomicAdd(&cnt[d], (uint32_t)__popcll(peers));
  __syncthreads();
  if (threadIdx.x < RADIX) ws.hist[(size_t)threadIdx.x * max_tiles + blockIdx.x] = cnt[threadIdx.x];
  if (threadIdx.x == 0) ws.tile_visible[blockIdx.x] = total;
}

void launch_preprocess(const gsr_gaussians &g, const gsr_camera *cams, const ViewInfo *views,
                       int n_views, const gsr_config &cfg, const Workspace &ws, bool clear_grad2d,
                       float *loss_zero, int max_sort_tiles, int order_total, hipStream_t s) {
  PreConsts pc{cfg.z_near, cfg.lowpass, cfg.cutoff_sigma, cfg.flags, cfg.fov_guard, cfg.alpha_min,
               clear_grad2d ? 1 : 0, loss_zero, order_total};
  const int64_t n_rec = g.n * (int64_t)n_views;
  if (g.n > 0) {
    hipLaunchKernelGGL(g.sh ? k_preprocess<true> : k_preprocess<false>, dim3((unsigned)((n_rec + PRE_BLOCK - 1) / PRE_BLOCK)), dim3(PRE_BLOCK), 0, s,
                       g, cams, views, pc, ws, n_views, max_sort_tiles);
  } else {
    launch_reset_header(ws, s);
    if (loss_zero) launch_fill_f32(loss_zero, 0.f, 1, s);
    launch_queue_order(ws, order_total, s);
  }
}

// Reliable-Gaussian selection (Eq. 12): compare each centre's camera depth
// with the observed depth at the nearest pixel.
__global__ __launch_bounds__(BLOCK) void k_select_reliable(gsr_gaussians g, const gsr_camera *__restrict__ cam,
                                                           const float *__restrict__ depth, int W, int H,
                                                           double eps, double z_near, uint8_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.n) return;
  uint8_t keep = 1;
  if (g.mask && g.mask[i] == 0) {
    keep = 0;
  } else {
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
        const double D = depth[(int64_t)pyd * W + (int64_t)pxd];
        if (D > 0.0 && fabs(D - z) > eps) keep = 0;
      }
    }
  }
  out[i] = keep;
}

void launch_select_reliable(const gsr_gaussians &g, const gsr_camera *cam, const float *depth, int W, int H,
                            float eps, float z_near, uint8_t *out, hipStream_t s) {
  if (g.n > 0)
    hipLaunchKernelGGL(k_select_reliable, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g, cam,
                       depth, W, H, (double)eps, (double)z_near, out);
}

}  // namespace gsr
