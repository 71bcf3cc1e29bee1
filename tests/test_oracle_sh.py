"""Pins of the oracle's degree-1 spherical-harmonic colour (Sec. 3.1: 12
coefficients per Gaussian, 4 per colour channel) and its gradients: the
basis against orthonormality on the sphere and a sign case, the viewing
direction against rigid-motion invariance, the backward against central
differences (coefficients, means, the se(3) pose and the paper's (q, t)
pose) and the translation gauge identity."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from oracle import splat as S
import workloads as W


def test_basis_is_orthonormal_on_the_sphere():
    """Gauss-Legendre in cos(theta) x uniform in phi integrates products of
    degree-1 harmonics exactly: the Gram matrix of the four basis functions
    is the identity."""
    ct, wt = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([np.outer(st, np.cos(phi)).ravel(), np.outer(st, np.sin(phi)).ravel(),
                  np.repeat(ct, nphi)], axis=1)
    w = np.repeat(wt, nphi) * (2 * np.pi / nphi)
    Y = S.sh_basis(d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(4), atol=1e-13)


def _one(pos, sh):
    return W.Scene(np.array([pos], np.float32), np.full((1, 3), math.log(0.05), np.float32),
                   np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), np.array([3.0], np.float32),
                   np.zeros((1, 3), np.float32), sh=np.asarray(sh, np.float32).reshape(1, 4, 3))


def test_sign_and_constant_term():
    """A Gaussian straight ahead of an identity camera (viewing direction
    +z): the z coefficient raises the colour, the x and y coefficients do not
    change it; with the constant coefficient only, the colour is that of the
    RGB model with rgb = Y_0 k_0 (the view-independent light version)."""
    cam = W.camera_small()
    base = np.zeros((4, 3))
    base[0] = [1.0, 2.0, 0.5]
    r0 = O.render(_one([0, 0, 2.0], base), cam)
    for k, sign in ((2, 1), (1, 0), (3, 0)):
        sh = base.copy()
        sh[k] = 0.3
        r = O.render(_one([0, 0, 2.0], sh), cam)
        d = r["rgb"][:, 60, 80] - r0["rgb"][:, 60, 80]
        assert (np.sign(np.round(d, 12)) == sign).all(), (k, d)
    rgb_scene = W.Scene(*(a.copy() for a in _one([0, 0, 2.0], base).arrays()))
    rgb_scene.rgb[:] = S.SH_C0 * base[0]
    np.testing.assert_allclose(r0["rgb"], O.render(rgb_scene, cam)["rgb"], atol=1e-14)


def _ham(p, q):
    w1, x1, y1, z1 = p.T
    w2, x2, y2, z2 = q.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def test_rigid_motion_with_rotated_coefficients_leaves_the_image_unchanged():
    """Move scene and camera by one rigid motion (R_w, t_w) and rotate each
    channel's degree-1 coefficient vector, read as the (x, y, z) vector
    (k_3, k_1, k_2), by R_w: every pixel is unchanged.  Fails if the viewing
    direction is not taken from the camera centre or the basis pairs a
    coefficient with the wrong axis."""
    sc = W.with_sh(W.random_scene(300, seed=8), seed=2)
    cam = W.perturb_pose(W.camera_small(), [0.1, -0.05, 0.2, 0.05, 0.1, -0.03])
    T = W.se3_exp([0.4, -0.3, 0.6, 0.5, -0.4, 0.3])
    Rw, tw = T[:3, :3], T[:3, 3]
    w = math.sqrt(1 + np.trace(Rw)) / 2
    qw = np.array([w, (Rw[2, 1] - Rw[1, 2]) / (4 * w), (Rw[0, 2] - Rw[2, 0]) / (4 * w), (Rw[1, 0] - Rw[0, 1]) / (4 * w)])
    sh = sc.sh.astype(float)
    vec = np.stack([sh[:, 3], sh[:, 1], sh[:, 2]], axis=1)  # [n, xyz, channel]
    vec2 = np.einsum("ij,njc->nic", Rw, vec)
    sh2 = sh.copy()
    sh2[:, 3], sh2[:, 1], sh2[:, 2] = vec2[:, 0], vec2[:, 1], vec2[:, 2]
    moved = W.Scene(sc.mean.astype(float) @ Rw.T + tw, sc.log_scale.astype(float),
                    _ham(np.tile(qw, (sc.n, 1)), sc.quat.astype(float)), sc.opacity_logit.astype(float),
                    sc.rgb.astype(float), sh=sh2)
    sc64 = W.Scene(*(a.astype(float) for a in sc.arrays()), sh=sh)
    R2 = np.asarray(cam.R, float) @ Rw.T
    t2 = np.asarray(cam.t, float) - R2 @ tw
    cam2 = dataclasses.replace(cam, R=R2, t=t2)
    r1, r2 = O.render(sc64, dataclasses.replace(cam, R=np.asarray(cam.R, float), t=np.asarray(cam.t, float))), \
        O.render(moved, cam2)
    ok = ~(r1["ambiguous"] | r2["ambiguous"])
    assert np.abs(r1["rgb"]).max() > 0.1
    np.testing.assert_allclose(r1["rgb"][:, ok], r2["rgb"][:, ok], atol=1e-9)
    # without rotating the coefficients the colours change
    r3 = O.render(dataclasses.replace(moved, sh=sh), cam2)
    assert np.abs(r3["rgb"][:, ok] - r1["rgb"][:, ok]).max() > 1e-3


def _fd_setup():
    rng = np.random.default_rng(31)
    n = 5
    mean = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), np.linspace(1.6, 3.4, n)], 1)
    sc = W.Scene(mean, np.log(0.18) + rng.normal(0, 0.3, (n, 3)), rng.normal(size=(n, 4)),
                 rng.uniform(-1.0, 1.5, n), np.zeros((n, 3)),
                 sh=np.concatenate([rng.uniform(0.5, 1.5, (n, 1, 3)), rng.normal(0, 0.5, (n, 3, 3))], axis=1))
    T = W.se3_exp([0.3, -0.2, 0.4, 0.2, -0.3, 0.25])  # a strongly rotated, offset camera
    cam = W.Camera(22.0, 22.0, 11.5, 9.5, T[:3, :3], T[:3, 3], 24, 20)
    cam = dataclasses.replace(cam, R=T[:3, :3], t=T[:3, 3])
    # keep the Gaussians in front of the camera: place them along its view
    R, t = T[:3, :3], T[:3, 3]
    sc = dataclasses.replace(sc, mean=(sc.mean - t) @ R)
    wts = (rng.normal(size=(3, 20, 24)), rng.normal(size=(20, 24)), rng.normal(size=(20, 24)))
    return sc, cam, wts


def _obj(sc, cam, cfg, wts):
    r = O.render(sc, cam, cfg)
    return float(np.sum(wts[0] * r["rgb"]) + np.sum(wts[1] * r["depth"]) + np.sum(wts[2] * r["T_final"]))


def test_sh_backward_matches_central_differences():
    sc, cam, wts = _fd_setup()
    cfg = O.Config.smooth(bg=(0.3, 0.6, 0.9))
    g = O.render_backward(sc, cam, cfg, *wts)
    h = 1e-6
    assert "sh" in g and np.abs(g["sh"]).max() > 0
    for name in ("sh", "mean"):
        arr = getattr(sc, name)
        flat = arr.reshape(arr.shape[0], -1)
        an = g[name].reshape(flat.shape)
        for i in range(flat.shape[0]):
            for j in range(flat.shape[1]):
                orig = flat[i, j]
                flat[i, j] = orig + h
                lp = _obj(sc, cam, cfg, wts)
                flat[i, j] = orig - h
                lm = _obj(sc, cam, cfg, wts)
                flat[i, j] = orig
                fd = (lp - lm) / (2 * h)
                assert abs(fd - an[i, j]) <= 1e-6 * (1 + abs(fd)), (name, i, j, fd, an[i, j])
    T0 = np.block([[np.asarray(cam.R, float), np.asarray(cam.t, float)[:, None]], [np.zeros((1, 3)), np.ones((1, 1))]])
    for k in range(6):
        vals = []
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[k] = sgn * h
            T = W.se3_exp(xi) @ T0
            vals.append(_obj(sc, dataclasses.replace(cam, R=T[:3, :3], t=T[:3, 3]), cfg, wts))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g["pose"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, g["pose"][k])


def test_sh_quaternion_translation_gradient_matches_finite_differences():
    """The paper's (q, t) pose with SH colour: the viewing directions move
    with the camera centre -R(q)^T t."""
    sc, cam, wts = _fd_setup()
    cfg = O.Config.smooth(bg=(0.3, 0.6, 0.9)).as_f32()
    R = np.asarray(cam.R, float)
    w = math.sqrt(1 + np.trace(R)) / 2
    q = np.array([w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w), (R[1, 0] - R[0, 1]) / (4 * w)]) * 1.3
    t = np.asarray(cam.t, float)

    def cam_qt(qq, tt):
        Rq, tq = O.pose_from_qt(qq, tt)
        return dataclasses.replace(cam, R=Rq, t=tq)

    c0 = cam_qt(q, t)
    g = O.render_backward(sc, c0, cfg, *wts)
    b = O.backward_params(g["fwd"]["proj"], g["grad2d"], cfg, pose_q=q)
    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd = (_obj(sc, cam_qt(q + e, t), cfg, wts) - _obj(sc, cam_qt(q - e, t), cfg, wts)) / (2 * h)
        assert abs(fd - b["pose_q"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, b["pose_q"][k])
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (_obj(sc, cam_qt(q, t + e), cfg, wts) - _obj(sc, cam_qt(q, t - e), cfg, wts)) / (2 * h)
        assert abs(fd - b["pose_t"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, b["pose_t"][k])


def test_sh_translation_gauge_identity():
    """Moving the camera by rho equals moving every mean by R^T rho, also
    through the viewing directions: dL/drho = R sum_i dL/dmu_i."""
    sc = W.with_sh(W.random_scene(800, seed=12), seed=3)
    cam = W.perturb_pose(W.camera_small(), [0.05, -0.02, 0.1, 0.02, 0.03, -0.01])
    gr, gd, gt = W.upstream_grads([(cam.width, cam.height)], seed=5)
    g = O.render_backward(sc, cam, O.Config(), gr.reshape(3, 120, 160), gd.reshape(120, 160), gt.reshape(120, 160))
    lhs = g["pose"][:3]
    rhs = np.asarray(cam.R, float) @ g["mean"].sum(0)
    np.testing.assert_allclose(lhs, rhs, rtol=5e-7, atol=5e-7 * np.abs(lhs).max())
    # the viewing-direction path matters: dropping it breaks the identity
    proj = g["fwd"]["proj"]
    b = O.backward_params({k: v for k, v in proj.items() if not k.startswith("sh")}, g["grad2d"], O.Config())
    assert np.abs(b["pose"][:3] - lhs).max() > 1e-4 * np.abs(lhs).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_sh_gradient_of_the_coefficients_is_basis_times_colour_gradient(seed):
    """The image is linear in the coefficients: the backward's coefficient
    gradient equals the linear map's transpose, found by rendering with one
    coefficient at 1 and the others at 0 (superposition)."""
    sc = W.with_sh(W.random_scene(60, seed=seed), seed=seed)
    cam = W.camera_small().with_size(40.0, 40.0, 15.5, 11.5, 32, 24)
    cfg = O.Config()
    wts = (np.random.default_rng(seed).normal(size=(3, 24, 32)), np.zeros((24, 32)), np.zeros((24, 32)))
    g = O.render_backward(sc, cam, cfg, *wts)
    for i in (0, 7, 33):
        for k in range(4):
            for c in range(3):
                unit = np.zeros_like(sc.sh)
                unit[i, k, c] = 1.0
                r = O.render(dataclasses.replace(sc, sh=unit), cam, cfg)
                assert abs(np.sum(wts[0] * r["rgb"]) - g["sh"][i, k, c]) <= 1e-9 * (1 + abs(g["sh"][i, k, c]))
