"""Pins of the oracle's pose parameterisations: the SE(3) exponential against
closed forms, its left Jacobian against finite differences of compositions,
and the gradient in the paper's quaternion + translation pose (supplement
Sec. A, eq. q2R, eq. grad_q) against FP64 central differences of the render
objective and against the printed derivative matrices."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.golden.load import evaluate, load_expressions

RNG = np.random.default_rng(77)


def test_se3_exp_closed_forms():
    # pure translation
    T = O.se3_exp([0.3, -0.2, 0.5, 0, 0, 0])
    np.testing.assert_allclose(T[:3, :3], np.eye(3), atol=1e-15)
    np.testing.assert_allclose(T[:3, 3], [0.3, -0.2, 0.5], atol=1e-15)
    # rotation by th about z, with the translation along the axis unchanged
    th = 0.7
    T = O.se3_exp([0.0, 0.0, 0.4, 0.0, 0.0, th])
    c, s = math.cos(th), math.sin(th)
    np.testing.assert_allclose(T[:3, :3], [[c, -s, 0], [s, c, 0], [0, 0, 1]], atol=1e-14)
    np.testing.assert_allclose(T[:3, 3], [0, 0, 0.4], atol=1e-14)
    for _ in range(5):
        xi = RNG.normal(size=6)
        T = O.se3_exp(xi)
        R = T[:3, :3]
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-13
        np.testing.assert_allclose(T @ O.se3_exp(-xi), np.eye(4), atol=1e-13)
        # rotation of a vector about the unit axis k by |phi| (Rodrigues' rotation formula)
        ang = np.linalg.norm(xi[3:])
        k = xi[3:] / ang
        v = RNG.normal(size=3)
        rod = v * math.cos(ang) + np.cross(k, v) * math.sin(ang) + k * (k @ v) * (1 - math.cos(ang))
        np.testing.assert_allclose(R @ v, rod, atol=1e-13)


@pytest.mark.parametrize("scale", [1e-9, 1e-3, 0.3, 1.5])
def test_left_jacobian_matches_finite_differences(scale):
    """For F(T) = sum_j w_j . (T p_j): the derivative of F(Exp(xi) T0) in xi
    equals J_l(xi)^T times the derivative of F(Exp(d) Exp(xi) T0) in d at
    d = 0, both by FP64 central differences."""
    xi = RNG.normal(size=6) * scale
    T0 = O.se3_exp(RNG.normal(size=6))
    P = RNG.normal(size=(5, 3))
    Wt = RNG.normal(size=(5, 3))

    def F(T):
        return float(np.sum(Wt * (P @ T[:3, :3].T + T[:3, 3])))

    h = 1e-6
    d_xi = np.zeros(6)
    g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        d_xi[k] = (F(O.se3_exp(xi + e) @ T0) - F(O.se3_exp(xi - e) @ T0)) / (2 * h)
        g[k] = (F(O.se3_exp(e) @ O.se3_exp(xi) @ T0) - F(O.se3_exp(-e) @ O.se3_exp(xi) @ T0)) / (2 * h)
    np.testing.assert_allclose(O.pose_xi_grad(xi, g), d_xi, rtol=1e-7, atol=1e-8)


def test_pose_from_qt_is_quaternion_conjugation():
    q = RNG.normal(size=4) * 2.0
    R, t = O.pose_from_qt(q, [1.0, 2.0, 3.0])
    qh = q / np.linalg.norm(q)
    w, v = qh[0], qh[1:]
    p = RNG.normal(size=3)
    # q p q* for a unit quaternion
    rot = p + 2 * w * np.cross(v, p) + 2 * np.cross(v, np.cross(v, p))
    np.testing.assert_allclose(R @ p, rot, atol=1e-14)
    np.testing.assert_allclose(t, [1.0, 2.0, 3.0])


def _fd_setup():
    rng = np.random.default_rng(21)
    n = 5
    mean = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), np.linspace(1.6, 3.4, n)], 1)
    sc = W.Scene(mean, np.log(0.18) + rng.normal(0, 0.3, (n, 3)), rng.normal(size=(n, 4)),
                 rng.uniform(-1.0, 1.5, n), rng.random((n, 3)))
    q = np.array([0.98, 0.05, -0.12, 0.1]) * 1.3   # not unit: the normalisation is part of the map
    t = np.array([0.03, -0.05, 0.08])
    wr = np.random.default_rng(3)
    wts = wr.normal(size=(3, 20, 24)), wr.normal(size=(20, 24)), wr.normal(size=(20, 24))
    return sc, q, t, wts


def _cam_qt(q, t):
    R, tt = O.pose_from_qt(q, t)
    return W.Camera(22.0, 22.0, 11.5, 9.5, R, tt, 24, 20)


def _obj(r, wts):
    return float(np.sum(wts[0] * r["rgb"]) + np.sum(wts[1] * r["depth"]) + np.sum(wts[2] * r["T_final"]))


@pytest.mark.parametrize("approx", [False, True])
def test_quaternion_translation_gradient_matches_finite_differences(approx):
    """Smooth mode, FP64 central differences in the 4 quaternion and 3
    translation components.  With approx_pose the screen covariance is held
    at its base-pose value (the dropped path of the paper)."""
    sc, q, t, wts = _fd_setup()
    cfg = O.Config.smooth(bg=(0.3, 0.6, 0.9)).as_f32()
    cam = _cam_qt(q, t)
    g = O.render_backward(sc, cam, cfg, *wts, approx_pose=approx, fwd=None)
    b = O.backward_params(g["fwd"]["proj"], g["grad2d"], cfg, approx_pose=approx, pose_q=q)
    base = O.project(sc, cam, cfg)

    def L(qq, tt):
        c2 = _cam_qt(qq, tt)
        p = dict(O.project(sc, c2, cfg))
        if approx:
            p["conic"], p["cov2"] = base["conic"], base["cov2"]
        return _obj(O.render(sc, c2, cfg, proj=p), wts)

    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd = (L(q + e, t) - L(q - e, t)) / (2 * h)
        assert abs(fd - b["pose_q"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, b["pose_q"][k])
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (L(q, t + e) - L(q, t - e)) / (2 * h)
        assert abs(fd - b["pose_t"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, b["pose_t"][k])
    # the translation gradient is the rho part of the left-perturbation gradient
    np.testing.assert_allclose(b["pose_t"], b["pose"][:3], rtol=1e-12, atol=1e-12)


def test_quaternion_gradient_centre_path_uses_the_printed_matrices():
    """The paper-approximate quaternion gradient (centres and depths only) is
    sum_i dL/dX_c,i . dX_c,i/dq with dX_c/dq the supplement's printed
    matrices (eq. grad_q, one sign corrected) at the world point, projected
    onto the tangent of the normalisation."""
    sc, q, t, wts = _fd_setup()
    cfg = O.Config.smooth().as_f32()
    cam = _cam_qt(q, t)
    g = O.render_backward(sc, cam, cfg, *wts, approx_pose=True)
    proj = g["fwd"]["proj"]
    b = O.backward_params(proj, g["grad2d"], cfg, approx_pose=True, pose_q=q)
    # dL/dX_c along centre and depth only, from the 2D gradients
    g2 = g["grad2d"]
    fx, fy = proj["fx"], proj["fy"]
    x, y, z = proj["Xc"].T
    gX = np.stack([g2[:, 0] * fx / z, g2[:, 1] * fy / z,
                   -g2[:, 0] * fx * x / z ** 2 - g2[:, 1] * fy * y / z ** 2 + g2[:, 9]], 1)
    table = load_expressions("dXc_dq.txt")
    qh = q / np.linalg.norm(q)
    gq = np.zeros(4)
    for i in range(sc.n):
        env = dict(qr=qh[0], qi=qh[1], qj=qh[2], qk=qh[3], x=sc.mean[i, 0], y=sc.mean[i, 1], z=sc.mean[i, 2])
        for k, name in enumerate(("q_r", "q_i", "q_j", "q_k")):
            dX = 2.0 * np.array(evaluate(table[name], env), dtype=float).sum(axis=1)
            gq[k] += gX[i] @ dX
    want = (gq - qh * (qh @ gq)) / np.linalg.norm(q)
    np.testing.assert_allclose(b["pose_q"], want, rtol=1e-10, atol=1e-12)
