// Camera-pose parameterisations around the renderer: the se(3) increment
// T = Exp(xi) T0 and the paper's quaternion + translation pose (supplement
// Sec. A: the pose is stored as a quaternion q and a translation t, R from
// eq. q2R).  The renderer's own pose gradient is the left-perturbation
// gradient g = (g_rho, g_phi) at the rendered pose; these kernels build the
// cameras from either parameterisation and chain g to it.  One thread per
// view, FP64 inside.
#pragma clang fp contract(off)

#include <math.h>

#include "gsr_internal.h"

namespace gsr {

namespace {

__device__ inline void hat(const double w[3], double K[9]) {
  K[0] = 0.0;   K[1] = -w[2]; K[2] = w[1];
  K[3] = w[2];  K[4] = 0.0;   K[5] = -w[0];
  K[6] = -w[1]; K[7] = w[0];  K[8] = 0.0;
}

__device__ inline void mat3_mul(const double A[9], const double B[9], double C[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[3 * r + c] = (A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c]) + A[3 * r + 2] * B[6 + c];
}

// Coefficients of the SO(3) / SE(3) closed forms in the rotation angle th
// (th2 = th^2): a = sin th / th, b = (1 - cos th) / th^2,
// c = (th - sin th) / th^3, d = (th^2 + 2 cos th - 2) / (2 th^4),
// e = (2 th - 3 sin th + th cos th) / (2 th^5).  Below th = 1e-2 the
// cancelling forms are replaced by their Taylor series (error < 1e-16
// relative there).
struct ExpCoef {
  double a, b, c, d, e;
};

__device__ inline ExpCoef exp_coef(double th2) {
  ExpCoef k;
  if (th2 < 1e-4) {
    k.a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    k.b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    k.c = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    k.d = 1.0 / 24.0 - th2 / 720.0 + th2 * th2 / 40320.0;
    k.e = 1.0 / 120.0 - th2 / 2520.0 + th2 * th2 / 120960.0;
  } else {
    const double th = sqrt(th2), s = sin(th), co = cos(th);
    k.a = s / th;
    k.b = (1.0 - co) / th2;
    k.c = (th - s) / (th2 * th);
    k.d = (th2 + 2.0 * co - 2.0) / (2.0 * th2 * th2);
    k.e = (2.0 * th - 3.0 * s + th * co) / (2.0 * th2 * th2 * th);
  }
  return k;
}

// Exp(xi) = [[R, V rho], [0, 1]] with R = I + a K + b K^2, V = I + b K + c K^2,
// K = hat(phi), xi = (rho, phi).
__device__ inline void se3_exp(const double xi[6], double R[9], double t[3]) {
  const double phi[3] = {xi[3], xi[4], xi[5]};
  double K[9], K2[9];
  hat(phi, K);
  mat3_mul(K, K, K2);
  const ExpCoef k = exp_coef((phi[0] * phi[0] + phi[1] * phi[1]) + phi[2] * phi[2]);
  double V[9];
  for (int j = 0; j < 9; ++j) {
    const double I = (j % 4 == 0) ? 1.0 : 0.0;
    R[j] = (I + k.a * K[j]) + k.b * K2[j];
    V[j] = (I + k.b * K[j]) + k.c * K2[j];
  }
  for (int r = 0; r < 3; ++r) t[r] = (V[3 * r] * xi[0] + V[3 * r + 1] * xi[1]) + V[3 * r + 2] * xi[2];
}

// Rotation of a unit quaternion (w, x, y, z), eq. q2R, and its derivatives
// w.r.t. the four components (for the chain through the normalisation).
__device__ inline void q2R(double w, double x, double y, double z, double R[9]) {
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline void q2R_grad(double w, double x, double y, double z, double D[4][9]) {
  const double d0[9] = {0.0, -z, y, z, 0.0, -x, -y, x, 0.0};
  const double d1[9] = {0.0, y, z, y, -2.0 * x, -w, z, w, -2.0 * x};
  const double d2[9] = {-2.0 * y, x, w, x, 0.0, z, -w, z, -2.0 * y};
  const double d3[9] = {-2.0 * z, -w, x, w, -2.0 * z, y, x, y, 0.0};
  for (int j = 0; j < 9; ++j) {
    D[0][j] = 2.0 * d0[j];
    D[1][j] = 2.0 * d1[j];
    D[2][j] = 2.0 * d2[j];
    D[3][j] = 2.0 * d3[j];
  }
}

__device__ inline void write_pose(gsr_camera &c, const double R[9], const double t[3]) {
  for (int j = 0; j < 9; ++j) c.R[j] = (float)R[j];
  for (int j = 0; j < 3; ++j) c.t[j] = (float)t[j];
}

}  // namespace

// cams_out[v] = cams_in[v] with the pose Exp(xi_v) (R_in, t_in).
__global__ void k_pose_apply(int n, const float *__restrict__ xi, const gsr_camera *__restrict__ cin,
                             gsr_camera *__restrict__ cout) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double x[6];
  for (int j = 0; j < 6; ++j) x[j] = xi[6 * v + j];
  double E[9], e[3];
  se3_exp(x, E, e);
  gsr_camera c = cin[v];
  double R0[9], R[9], t[3];
  for (int j = 0; j < 9; ++j) R0[j] = c.R[j];
  mat3_mul(E, R0, R);
  for (int r = 0; r < 3; ++r)
    t[r] = ((E[3 * r] * (double)c.t[0] + E[3 * r + 1] * (double)c.t[1]) + E[3 * r + 2] * (double)c.t[2]) + e[r];
  write_pose(c, R, t);
  cout[v] = c;
}

// d_xi = J_l(xi)^T d_pose with the SE(3) left Jacobian
//   J_l = [[J, Q], [0, J]],  J = I + b K + c K^2 (the SO(3) left Jacobian),
//   Q = rho^/2 + c (K P + P K + K P K) + d (K^2 P + P K^2 - 3 K P K)
//       + e (K P K^2 + K^2 P K),  P = hat(rho),
// so that Exp(xi + dxi) = Exp(J_l dxi) Exp(xi) to first order: a loss of
// T = Exp(xi) T0 then has gradient J_l^T g in xi, g its left-perturbation
// gradient at T.
__global__ void k_pose_xi_grad(int n, const float *__restrict__ xi, const float *__restrict__ d_pose,
                               float *__restrict__ d_xi) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double rho[3] = {xi[6 * v], xi[6 * v + 1], xi[6 * v + 2]};
  const double phi[3] = {xi[6 * v + 3], xi[6 * v + 4], xi[6 * v + 5]};
  double K[9], K2[9], P[9];
  hat(phi, K);
  hat(rho, P);
  mat3_mul(K, K, K2);
  const ExpCoef k = exp_coef((phi[0] * phi[0] + phi[1] * phi[1]) + phi[2] * phi[2]);
  double KP[9], PK[9], KPK[9], K2P[9], PK2[9], KPK2[9], K2PK[9];
  mat3_mul(K, P, KP);
  mat3_mul(P, K, PK);
  mat3_mul(KP, K, KPK);
  mat3_mul(K2, P, K2P);
  mat3_mul(P, K2, PK2);
  mat3_mul(KP, K2, KPK2);
  mat3_mul(K2, PK, K2PK);
  double J[9], Q[9];
  for (int j = 0; j < 9; ++j) {
    const double I = (j % 4 == 0) ? 1.0 : 0.0;
    J[j] = (I + k.b * K[j]) + k.c * K2[j];
    Q[j] = ((0.5 * P[j] + k.c * ((KP[j] + PK[j]) + KPK[j])) + k.d * ((K2P[j] + PK2[j]) - 3.0 * KPK[j])) +
           k.e * (KPK2[j] + K2PK[j]);
  }
  double g[6];
  for (int j = 0; j < 6; ++j) g[j] = d_pose[6 * v + j];
  // [J^T 0; Q^T J^T] g
  for (int c = 0; c < 3; ++c) {
    d_xi[6 * v + c] = (float)((J[c] * g[0] + J[3 + c] * g[1]) + J[6 + c] * g[2]);
    d_xi[6 * v + 3 + c] = (float)(((Q[c] * g[0] + Q[3 + c] * g[1]) + Q[6 + c] * g[2]) +
                                  ((J[c] * g[3] + J[3 + c] * g[4]) + J[6 + c] * g[5]));
  }
}

// cams_out[v] = cams_in[v] (intrinsics, size) with R = q2R(q / |q|), t.
__global__ void k_pose_from_qt(int n, const float *__restrict__ q, const float *__restrict__ t,
                               const gsr_camera *__restrict__ cin, gsr_camera *__restrict__ cout) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double w = q[4 * v], x = q[4 * v + 1], y = q[4 * v + 2], z = q[4 * v + 3];
  const double qn = sqrt(((w * w + x * x) + y * y) + z * z);
  w /= qn; x /= qn; y /= qn; z /= qn;
  double R[9];
  q2R(w, x, y, z, R);
  const double tt[3] = {t[3 * v], t[3 * v + 1], t[3 * v + 2]};
  gsr_camera c = cin[v];
  write_pose(c, R, tt);
  cout[v] = c;
}

// Gradient in (q, t) of a loss whose left-perturbation gradient at
// T = [q2R(q/|q|) | t] is g = (g_rho, g_phi).  Moving t alone is the
// perturbation rho = dt: d_t = g_rho.  Moving q changes R by dR = (dR/dq) dq,
// which is the perturbation phi = vee(dR R^T) with rho = t x phi (the
// translation stays): d_q_k = w_k . (g_phi + g_rho x t), w_k = vee((dR/dq_k)
// R^T), and through the normalisation d_q = (I - qh qh^T) d_qh / |q|.
__global__ void k_pose_qt_grad(int n, const float *__restrict__ q, const float *__restrict__ t,
                               const float *__restrict__ d_pose, float *__restrict__ d_q,
                               float *__restrict__ d_t) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double w = q[4 * v], x = q[4 * v + 1], y = q[4 * v + 2], z = q[4 * v + 3];
  const double qn = sqrt(((w * w + x * x) + y * y) + z * z);
  w /= qn; x /= qn; y /= qn; z /= qn;
  double R[9], D[4][9];
  q2R(w, x, y, z, R);
  q2R_grad(w, x, y, z, D);
  const double gr[3] = {d_pose[6 * v], d_pose[6 * v + 1], d_pose[6 * v + 2]};
  const double tt[3] = {t[3 * v], t[3 * v + 1], t[3 * v + 2]};
  // s = g_phi + g_rho x t
  const double s[3] = {d_pose[6 * v + 3] + (gr[1] * tt[2] - gr[2] * tt[1]),
                       d_pose[6 * v + 4] + (gr[2] * tt[0] - gr[0] * tt[2]),
                       d_pose[6 * v + 5] + (gr[0] * tt[1] - gr[1] * tt[0])};
  double gq[4];
  for (int k = 0; k < 4; ++k) {
    double Rt[9], M[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Rt[3 * r + c] = R[3 * c + r];
    mat3_mul(D[k], Rt, M);
    // vee of the skew part of M: for a change of the unit quaternion along
    // its sphere the M_k dq_k sum to a skew matrix, so their skew parts give
    // the rotation exactly; the radial direction is projected out below.
    const double wv[3] = {0.5 * (M[7] - M[5]), 0.5 * (M[2] - M[6]), 0.5 * (M[3] - M[1])};
    gq[k] = (wv[0] * s[0] + wv[1] * s[1]) + wv[2] * s[2];
  }
  const double qh[4] = {w, x, y, z};
  const double dot = ((qh[0] * gq[0] + qh[1] * gq[1]) + qh[2] * gq[2]) + qh[3] * gq[3];
  for (int k = 0; k < 4; ++k) d_q[4 * v + k] = (float)((gq[k] - qh[k] * dot) / qn);
  for (int k = 0; k < 3; ++k) d_t[3 * v + k] = (float)gr[k];
}

void launch_pose_apply(int n, const float *xi, const gsr_camera *cin, gsr_camera *cout, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pose_apply, dim3((n + 63) / 64), dim3(64), 0, s, n, xi, cin, cout);
}

void launch_pose_xi_grad(int n, const float *xi, const float *d_pose, float *d_xi, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pose_xi_grad, dim3((n + 63) / 64), dim3(64), 0, s, n, xi, d_pose, d_xi);
}

void launch_pose_from_qt(int n, const float *q, const float *t, const gsr_camera *cin, gsr_camera *cout,
                         hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pose_from_qt, dim3((n + 63) / 64), dim3(64), 0, s, n, q, t, cin, cout);
}

void launch_pose_qt_grad(int n, const float *q, const float *t, const float *d_pose, float *d_q, float *d_t,
                         hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pose_qt_grad, dim3((n + 63) / 64), dim3(64), 0, s, n, q, t, d_pose, d_q, d_t);
}

}  // namespace gsr
