"""Camera-pose parameterisations in the CPU FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/splat.py): never imported by the
product path.

The renderer's pose gradient is the derivative w.r.t. a left perturbation
T <- Exp(xi) T at xi = 0 (Sec. 3.3, Eq. 11; supplement Sec. A).  Callers
parameterise the pose either as an se(3) increment on a base pose,
T = Exp(xi) T0, or as the paper stores it, a quaternion q and a translation t
with R = R(q / |q|) from eq. q2R (supplement Sec. A).  This module holds the
definitions those parameterisations need: the SE(3) exponential as the matrix
exponential of the twist, the left Jacobian as its power series, and the
cameras they give.  The (q, t) gradient itself is summed per Gaussian in
splat.backward_params (pose_q), through the derivatives of the camera-frame
points and covariances w.r.t. q and t, as the supplement derives it.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .splat import quat_to_rotmat


def hat(w):
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """Exp(xi) for xi = (rho, phi): the matrix exponential of the twist
    [[hat(phi), rho], [0, 0]] (4x4, FP64)."""
    xi = np.asarray(xi, np.float64)
    A = np.zeros((4, 4))
    A[:3, :3] = hat(xi[3:])
    A[:3, 3] = xi[:3]
    return scipy.linalg.expm(A)


def se3_left_jacobian(xi, tol=1e-18):
    """Left Jacobian of SE(3) at xi = (rho, phi): sum_k ad(xi)^k / (k + 1)!
    with ad(xi) = [[hat(phi), hat(rho)], [0, hat(phi)]] (6x6), summed until
    the terms fall below `tol` relative.  To first order
    Exp(xi + d) = Exp(J d) Exp(xi)."""
    xi = np.asarray(xi, np.float64)
    ad = np.zeros((6, 6))
    ad[:3, :3] = hat(xi[3:])
    ad[:3, 3:] = hat(xi[:3])
    ad[3:, 3:] = hat(xi[3:])
    J = np.eye(6)
    term = np.eye(6)
    for k in range(1, 200):
        term = term @ ad / (k + 1)
        J = J + term
        if np.abs(term).max() <= tol * np.abs(J).max():
            break
    return J


def pose_xi_grad(xi, g):
    """Gradient in xi of a loss of T = Exp(xi) T0 whose left-perturbation
    gradient at T is g: J_l(xi)^T g."""
    return se3_left_jacobian(xi).T @ np.asarray(g, np.float64)


def apply_xi(xi, R0, t0):
    """(R, t) of Exp(xi) [R0 | t0]."""
    T0 = np.eye(4)
    T0[:3, :3] = np.asarray(R0, np.float64).reshape(3, 3)
    T0[:3, 3] = np.asarray(t0, np.float64).reshape(3)
    T = se3_exp(xi) @ T0
    return T[:3, :3], T[:3, 3]


def pose_from_qt(q, t):
    """World->camera (R, t) of the paper's pose: R = R(q / |q|) (eq. q2R)."""
    q = np.asarray(q, np.float64).reshape(1, 4)
    qh = q / math.sqrt(float((q * q).sum()))
    return quat_to_rotmat(qh)[0], np.asarray(t, np.float64).reshape(3)
