"""Adaptive expansion of the Gaussian map in the CPU FP64 oracle (GS-SLAM
Sec. 3.2, Eq. 8 adding step, Eq. 9 deleting step).

TEST INFRASTRUCTURE ONLY (see oracle/splat.py): never imported by the
product path.

Adding step (Eq. 8).  After rendering a keyframe, a pixel is unreliable when
its cumulative opacity A = 1 - T_final is below tau_T or its rendered depth
D_hat is farther than tau_D from the observed depth D.  Unreliable pixels
are back-projected with their observed depth and each becomes a new Gaussian
initialised as at map initialisation (Eq. 7): position the back-projected
point, colour the observed colour, a predefined opacity, and an isotropic
covariance set by the point density.  Readings (the paper is silent):
  * a pixel without a depth reading (D = 0) cannot be back-projected and is
    never added;
  * the decisions are taken in FP64 on the float32 inputs;
  * the new Gaussians are appended in pixel order (views in order, rows top to
    bottom, pixels left to right);
  * the density-dependent scale is the spacing of back-projected neighbouring
    pixels on a fronto-parallel surface, D / sqrt(fx fy), times a factor; the
    rotation is the identity quaternion;
  * in a map with degree-1 spherical-harmonic colour (Sec. 3.1) the new
    Gaussian's coefficients are the ones whose colour is the observed colour
    from every direction: the constant term colour / Y_0, the three linear
    terms zero.

Deleting step (Eq. 9).  Each visible Gaussian's ray from the camera centre
through its centre X_i meets the image at a pixel with observed depth D; the
world point P_uv of that pixel at its observed depth lies on the same ray.
The printed condition D - dist(X_i, P_uv) > gamma is garbled: read literally
it would decay Gaussians lying on the surface (dist = 0).  The prose says the
opacity of Gaussians floating in front of the surface is decreased, so the
reading is: the signed distance along the ray from X_i to P_uv,
(D - z) |X_c| / z (positive when the observed surface lies beyond the
Gaussian), exceeds gamma.  "Visible" means z > z_near and the projected
centre's nearest pixel inside the image; the pixel must hold a reading
(D > 0).  The decay scales the opacity itself, sigmoid(Lambda') =
eta sigmoid(Lambda) (scaling the logit would move a low opacity towards 0.5).
"""
from __future__ import annotations

import math

import numpy as np

from .splat import SH_C0

F64 = np.float64


def adding_mask(T_final, depth, depth_obs, tau_T, tau_D):
    """Eq. 8 per pixel: D > 0 and (1 - T_final < tau_T or |D - D_hat| > tau_D),
    in FP64 on the float32 values.  Arrays of one shape; returns bool."""
    T = np.asarray(T_final, np.float32).astype(F64)
    Dh = np.asarray(depth, np.float32).astype(F64)
    D = np.asarray(depth_obs, np.float32).astype(F64)
    tT = float(np.float32(tau_T))
    tD = float(np.float32(tau_D))
    with np.errstate(invalid="ignore"):
        return (D > 0.0) & (((1.0 - T) < tT) | (np.abs(D - Dh) > tD))


def back_project(x, y, D, cam):
    """World point of pixel (x, y) at camera-frame depth D (pixel centres at
    integer coordinates): X_c = (D (x - cx) / fx, D (y - cy) / fy, D) and
    X = R^T (X_c - t) for the world->camera pose X_c = R X + t."""
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    R = np.asarray(cam.R, np.float32).astype(F64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(F64).reshape(3)
    Xc = np.array([D * (x - cx) / fx, D * (y - cy) / fy, D], F64)
    return R.T @ (Xc - t)


def add_gaussians(cams, T_final, depth, depth_obs, rgb_obs, tau_T, tau_D, scale_factor, opacity_logit_init):
    """The adding step over views (lists of per-view arrays: T_final, depth,
    depth_obs [H, W], rgb_obs [3, H, W]).  Returns (mask per view, dict of the
    new Gaussians in pixel order: mean [m, 3], log_scale [m, 3], quat [m, 4],
    opacity_logit [m], rgb [m, 3], sh [m, 4, 3] (for a spherical-harmonic
    map), pixel [m, 3] = (view, x, y))."""
    masks = []
    parts = dict(mean=[], log_scale=[], rgb=[], pixel=[])
    for v, cam in enumerate(cams):
        m = adding_mask(T_final[v], depth[v], depth_obs[v], tau_T, tau_D)
        masks.append(m)
        fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
        Dobs = np.asarray(depth_obs[v], np.float32)
        C = np.asarray(rgb_obs[v], np.float32).reshape(3, *Dobs.shape)
        ys, xs = np.nonzero(m)  # row-major order
        for x, y in zip(xs.tolist(), ys.tolist()):
            D = float(Dobs[y, x])
            parts["mean"].append(back_project(x, y, D, cam))
            s = float(np.float32(scale_factor)) * D / math.sqrt(fx * fy)
            parts["log_scale"].append([math.log(s)] * 3)
            parts["rgb"].append(C[:, y, x].astype(F64))
            parts["pixel"].append((v, x, y))
    k = len(parts["mean"])
    out = dict(mean=np.array(parts["mean"], F64).reshape(k, 3),
               log_scale=np.array(parts["log_scale"], F64).reshape(k, 3),
               quat=np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (k, 1)),
               opacity_logit=np.full(k, float(np.float32(opacity_logit_init))),
               rgb=np.array(parts["rgb"], F64).reshape(k, 3),
               pixel=np.array(parts["pixel"], np.int64).reshape(k, 3))
    sh = np.zeros((k, 4, 3), F64)
    sh[:, 0, :] = out["rgb"] / SH_C0
    out["sh"] = sh
    return masks, out


def delete_gaussians(mean, opacity_logit, cam, depth_obs, gamma, eta, z_near=0.2, mask=None):
    """The deleting step (Eq. 9, reading above) for one view.  Returns
    (new opacity logits [n] FP64, decayed [n] bool).  Gaussians excluded by
    `mask` are left alone."""
    mean = np.asarray(mean, np.float32).astype(F64)
    lam = np.asarray(opacity_logit, np.float32).astype(F64)
    R = np.asarray(cam.R, np.float32).astype(F64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(F64).reshape(3)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    Dimg = np.asarray(depth_obs, np.float32).reshape(int(cam.height), int(cam.width))
    g, e, zn = float(np.float32(gamma)), float(np.float32(eta)), float(np.float32(z_near))
    out = lam.copy()
    decayed = np.zeros(mean.shape[0], bool)
    for i in range(mean.shape[0]):  # one Gaussian at a time
        if mask is not None and not mask[i]:
            continue
        mx, my, mz = mean[i]
        x = ((R[0, 0] * mx + R[0, 1] * my) + R[0, 2] * mz) + t[0]
        y = ((R[1, 0] * mx + R[1, 1] * my) + R[1, 2] * mz) + t[1]
        z = ((R[2, 0] * mx + R[2, 1] * my) + R[2, 2] * mz) + t[2]
        if not z > zn:
            continue
        u = (fx * x) / z + cx
        v = (fy * y) / z + cy
        px, py = math.floor(u + 0.5), math.floor(v + 0.5)
        if not (0 <= px < int(cam.width) and 0 <= py < int(cam.height)):
            continue
        D = float(Dimg[py, px])
        if not D > 0.0:
            continue
        # P_uv = (D / z) X_c on the same ray; signed distance from X_i to it.
        s = (D - z) * math.sqrt((x * x + y * y) + z * z) / z
        if s > g:
            o = 1.0 / (1.0 + math.exp(-lam[i]))
            o2 = e * o
            out[i] = math.log(o2 / (1.0 - o2))
            decayed[i] = True
    return out, decayed
