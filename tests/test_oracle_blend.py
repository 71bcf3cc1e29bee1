"""Pins of the oracle's compositing (Eq. 4-5), its backward pass (supplement
eq. grad_depth and the chain through Eq. 3), the se(3) pose gradient and the
L1 loss: closed forms, a sequential per-pixel definition, invariants and FP64
central finite differences."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _scene(rows):
    """rows: (mean xyz, log_scale xyz, quat wxyz, opacity_logit, rgb)."""
    cols = list(zip(*rows))
    return W.Scene(*(np.array(c, np.float64) for c in cols))


def _cam(width, height, f, R=None, t=None):
    R = np.eye(3) if R is None else R
    t = np.zeros(3) if t is None else t
    return W.Camera(float(f), float(f), (width - 1) / 2, (height - 1) / 2, np.asarray(R, float),
                    np.asarray(t, float), width, height)


def test_single_gaussian_closed_form():
    # On the optical axis an isotropic Gaussian projects to an isotropic one:
    # Sigma' = (f s / z)^2 I + lowpass I, centred on the principal point.
    cam = dataclasses.replace(_cam(48, 40, 60.0), cx=20.3, cy=13.7)
    s, z, op = 0.05, 2.0, 0.8
    sc = _scene([((0.0, 0.0, z), (math.log(s),) * 3, (0.6, 0.0, 0.8, 0.0), op, (0.9, 0.2, 0.4))])
    cfg = O.Config(bg=(0.25, 0.5, 0.75)).as_f32()
    r = O.render(sc, cam, cfg)
    sig2 = (cam.fx * s / z) ** 2 + cfg.lowpass
    u, v = cam.cx, cam.cy
    p = r["proj"]
    tx0, tx1, ty0, ty1 = p["rect"][0]
    o = 1 / (1 + math.exp(-op))
    bg = np.array(cfg.bg)
    for py in range(cam.height):
        for px in range(cam.width):
            in_list = tx0 <= px // 16 <= tx1 and ty0 <= py // 16 <= ty1
            q = ((u - px) ** 2 + (v - py) ** 2) / sig2
            a = min(cfg.alpha_max, o * math.exp(-0.5 * q))
            if not in_list or a < cfg.alpha_min:
                a = 0.0
            np.testing.assert_allclose(r["rgb"][:, py, px], a * np.array([0.9, 0.2, 0.4]) + (1 - a) * bg,
                                       atol=1e-12)
            assert abs(r["depth"][py, px] - a * z) < 1e-12
            assert abs(r["T_final"][py, px] - (1 - a)) < 1e-12


def test_two_coaxial_gaussians():
    cam = _cam(32, 32, 50.0)
    z1, z2 = 1.5, 3.0
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.7])
    # Same projected centre: the far one is the near one scaled along the ray.
    m1 = np.array([0.02, 0.01, z1])
    m2 = m1 * (z2 / z1)
    sc = _scene([(tuple(m2), (math.log(0.06),) * 3, (1, 0, 0, 0), 1.0, tuple(c2)),
                 (tuple(m1), (math.log(0.03),) * 3, (1, 0, 0, 0), 0.5, tuple(c1))])
    cfg = O.Config().as_f32()
    r = O.render(sc, cam, cfg)
    p = r["proj"]
    np.testing.assert_allclose(p["uv"][0], p["uv"][1], atol=1e-12)
    u, v = p["uv"][1]
    for (py, px) in [(15, 15), (16, 16), (14, 17), (17, 14), (13, 18)]:
        al = []
        for k in (1, 0):  # near first
            a_, b_, c_ = p["conic"][k]
            dx, dy = u - px, v - py
            q = a_ * dx * dx + 2 * b_ * dx * dy + c_ * dy * dy
            al.append(min(cfg.alpha_max, p["opacity"][k] * math.exp(-0.5 * q)))
        a1, a2 = al
        assert min(al) >= cfg.alpha_min and (1 - a1) * (1 - a2) >= cfg.T_min
        np.testing.assert_allclose(r["rgb"][:, py, px], c1 * a1 + c2 * a2 * (1 - a1), atol=1e-12)
        assert abs(r["depth"][py, px] - (z1 * a1 + z2 * a2 * (1 - a1))) < 1e-12
        assert abs(r["T_final"][py, px] - (1 - a1) * (1 - a2)) < 1e-12


def _sequential_pixel(proj, lst, px, py, cfg):
    """The blending definition written as the per-pixel loop it describes."""
    T, C, D, last = 1.0, np.zeros(3), 0.0, 0
    for pos, i in enumerate(lst):
        a_, b_, c_ = proj["conic"][i]
        dx = proj["uv"][i, 0] - px
        dy = proj["uv"][i, 1] - py
        q = a_ * dx * dx + 2 * b_ * dx * dy + c_ * dy * dy
        alpha = min(cfg.alpha_max, proj["opacity"][i] * math.exp(-0.5 * q))
        if alpha < cfg.alpha_min:
            continue
        Tn = T * (1 - alpha)
        if Tn < cfg.T_min:
            break
        C += alpha * T * proj["rgb"][i]
        D += alpha * T * proj["z"][i]
        T = Tn
        last = pos + 1
    return C + T * np.asarray(cfg.bg), D, T, last


@pytest.mark.parametrize("seed", [0, 1])
def test_blend_matches_sequential_definition(seed):
    cam = _cam(40, 35, 45.0)
    sc = W.random_scene(500, seed=seed, xy=0.6, log_scale_mu=-2.3)
    sc.opacity_logit += 2.5  # dense and opaque: many pixels terminate early
    cfg = O.Config(bg=(0.1, 0.2, 0.3)).as_f32()
    r = O.render(sc, cam, cfg)
    p = r["proj"]
    starts, gauss = r["lists"]
    n_term = 0
    for py in range(cam.height):
        for px in range(cam.width):
            tile = (py // 16) * p["TX"] + px // 16
            lst = gauss[starts[tile]:starts[tile + 1]]
            C, D, T, last = _sequential_pixel(p, lst, px, py, cfg)
            np.testing.assert_allclose(r["rgb"][:, py, px], C, atol=1e-12)
            assert abs(r["depth"][py, px] - D) < 1e-12
            assert abs(r["T_final"][py, px] - T) < 1e-14
            assert r["last"][py, px] == last
            n_term += T < 2 * cfg.T_min
    assert n_term > 0  # the termination rule was exercised


def test_invariants_on_small_workload():
    sc = W.random_scene(2000, seed=0)
    cam = W.camera_small()
    cfg = O.Config().as_f32()
    r = O.render(sc, cam, cfg)
    A = 1 - r["T_final"]
    assert np.all(A >= 0) and np.all(A <= 1)
    # Telescoping: with every colour 1 and bg 0 the colour equals 1 - T_final.
    white = dataclasses.replace(sc, rgb=np.ones_like(sc.rgb))
    rw = O.render(white, cam, cfg)
    np.testing.assert_allclose(rw["rgb"][0], 1 - rw["T_final"], atol=1e-12)
    # Depth over accumulated opacity lies within the depth range of the tile list.
    p = r["proj"]
    starts, gauss = r["lists"]
    for tile in range(p["TX"] * p["TY"]):
        lst = gauss[starts[tile]:starts[tile + 1]]
        if lst.size == 0:
            continue
        ty, tx = divmod(tile, p["TX"])
        sl = (slice(ty * 16, ty * 16 + 16), slice(tx * 16, tx * 16 + 16))
        a_ = A[sl]
        ok = a_ > 1e-9
        dn = r["depth"][sl][ok] / a_[ok]
        zs = p["z"][lst]
        assert np.all(dn >= zs.min() - 1e-9) and np.all(dn <= zs.max() + 1e-9)
        cmax = np.maximum(sc.rgb[lst].max(0), 0.0)
        for ch in range(3):
            assert np.all(r["rgb"][ch][sl] <= cmax[ch] + 1e-9)
    assert r["ambiguous"].mean() < 2e-3


def test_input_order_invariance():
    sc = W.random_scene(600, seed=4)
    cam = W.camera_small()
    perm = np.random.default_rng(0).permutation(600)
    r1 = O.render(sc, cam)
    r2 = O.render(W.subset(sc, perm), cam)
    z = r1["proj"]["zbits"][r1["proj"]["valid"]]
    assert np.unique(z).size == z.size  # no depth ties, so the order is unique
    for k in ("rgb", "depth", "T_final"):
        np.testing.assert_allclose(r1[k], r2[k], atol=1e-13)


def test_rigid_motion_invariance():
    sc = W.random_scene(400, seed=6)
    cam = W.camera_small()
    T = W.se3_exp([0.3, -0.2, 0.5, 0.4, -0.3, 0.2])
    Rw, tw = T[:3, :3], T[:3, 3]
    # Move the scene by (Rw, tw) and the camera by the inverse motion.
    from oracle.splat import quat_to_rotmat
    qw = np.array([1.0, 0, 0, 0])
    # quaternion of Rw (Shepperd-free: Rw is a small rotation, w > 0)
    w = math.sqrt(max(0.0, 1 + np.trace(Rw))) / 2
    qw = np.array([w, (Rw[2, 1] - Rw[1, 2]) / (4 * w), (Rw[0, 2] - Rw[2, 0]) / (4 * w), (Rw[1, 0] - Rw[0, 1]) / (4 * w)])
    np.testing.assert_allclose(quat_to_rotmat(qw[None])[0], Rw, atol=1e-12)

    def ham(p, q):
        w1, x1, y1, z1 = p.T
        w2, x2, y2, z2 = q.T
        return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)

    q64 = sc.quat.astype(float)
    moved = W.Scene(sc.mean.astype(float) @ Rw.T + tw, sc.log_scale.astype(float),
                    ham(np.tile(qw, (400, 1)), q64), sc.opacity_logit.astype(float), sc.rgb.astype(float))
    R2 = np.asarray(cam.R, float) @ Rw.T
    t2 = np.asarray(cam.t, float) - R2 @ tw
    cam2 = dataclasses.replace(cam, R=R2, t=t2)
    r1 = O.render(sc, cam)
    r2 = O.render(moved, cam2)
    ok = ~(r1["ambiguous"] | r2["ambiguous"])
    for k in ("rgb", "depth", "T_final"):
        np.testing.assert_allclose(r1[k][..., ok], r2[k][..., ok], atol=1e-9)


# --------------------------------------------------------------------------- backward

def _fd_scene():
    rng = np.random.default_rng(21)
    n = 5
    mean = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), np.linspace(1.6, 3.4, n)], 1)
    ls = np.log(0.18) + rng.normal(0, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    op = rng.uniform(-1.0, 1.5, n)
    rgb = rng.random((n, 3))
    return W.Scene(mean, ls, q, op, rgb)


def _fd_cam():
    T = W.se3_exp([0.02, -0.03, 0.05, 0.03, -0.02, 0.04])
    return _cam(24, 20, 22.0, T[:3, :3], T[:3, 3])


def _weights(cam, seed=3):
    rng = np.random.default_rng(seed)
    H, Wd = cam.height, cam.width
    return rng.normal(size=(3, H, Wd)), rng.normal(size=(H, Wd)), rng.normal(size=(H, Wd))


def _objective(sc, cam, cfg, wts):
    r = O.render(sc, cam, cfg)
    return float(np.sum(wts[0] * r["rgb"]) + np.sum(wts[1] * r["depth"]) + np.sum(wts[2] * r["T_final"]))


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.3, 0.6, 0.9)])
def test_backward_matches_central_differences(bg):
    sc, cam = _fd_scene(), _fd_cam()
    cfg = O.Config.smooth(bg=bg)
    wts = _weights(cam)
    g = O.render_backward(sc, cam, cfg, *wts)
    h = 1e-6
    names = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
    for name in names:
        arr = getattr(sc, name)
        flat = arr.reshape(arr.shape[0], -1)
        an = g[name].reshape(flat.shape)
        for i in range(flat.shape[0]):
            for j in range(flat.shape[1]):
                orig = flat[i, j]
                flat[i, j] = orig + h
                lp = _objective(sc, cam, cfg, wts)
                flat[i, j] = orig - h
                lm = _objective(sc, cam, cfg, wts)
                flat[i, j] = orig
                fd = (lp - lm) / (2 * h)
                assert abs(fd - an[i, j]) <= 1e-6 * (1 + abs(fd)), (name, i, j, fd, an[i, j])
    for k in range(6):
        xi = np.zeros(6)
        vals = []
        for sgn in (1, -1):
            xi[k] = sgn * h
            T = W.se3_exp(xi) @ np.block([[np.asarray(cam.R, float), np.asarray(cam.t, float)[:, None]],
                                          [np.zeros((1, 3)), np.ones((1, 1))]])
            vals.append(_objective(sc, dataclasses.replace(cam, R=T[:3, :3], t=T[:3, 3]), cfg, wts))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g["pose"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, g["pose"][k])


def test_backward_matches_central_differences_outside_the_guard():
    """Two Gaussians whose x/z (resp. y/z) lies beyond the Jacobian guard
    but whose footprint reaches into the image: the limited Jacobian is
    differentiated exactly (no x dependence, 1/z dependence only)."""
    base = _fd_scene()
    extra = W.Scene(np.array([[0.8 * 2.0, 0.1, 2.0], [-0.2, 0.7 * 2.3, 2.3]]),
                    np.full((2, 3), np.log(0.25)), np.array([[0.9, 0.1, -0.3, 0.2], [0.5, -0.5, 0.5, 0.4]]),
                    np.array([1.2, 0.8]), np.array([[0.9, 0.2, 0.1], [0.1, 0.8, 0.3]]))
    sc = W.Scene(*(np.concatenate([a, b]) for a, b in zip(base.arrays(), extra.arrays())))
    cam = _cam(24, 20, 22.0)
    cfg = O.Config.smooth()
    p = O.project(sc, cam, cfg)
    assert not p["free_x"][5] and not p["free_y"][6] and p["free_x"][:5].all() and p["free_y"][:5].all()
    wts = _weights(cam)
    g = O.render_backward(sc, cam, cfg, *wts)
    h = 1e-6
    for name in ("mean", "log_scale"):
        arr = getattr(sc, name)
        for i in (5, 6):
            for j in range(3):
                orig = arr[i, j]
                arr[i, j] = orig + h
                lp = _objective(sc, cam, cfg, wts)
                arr[i, j] = orig - h
                lm = _objective(sc, cam, cfg, wts)
                arr[i, j] = orig
                fd = (lp - lm) / (2 * h)
                assert abs(g[name][i, j]) > 1e-4
                assert abs(fd - g[name][i, j]) <= 1e-6 * (1 + abs(fd)), (name, i, j, fd, g[name][i, j])
    for k in range(6):
        xi = np.zeros(6)
        vals = []
        for sgn in (1, -1):
            xi[k] = sgn * h
            T = W.se3_exp(xi)
            vals.append(_objective(sc, dataclasses.replace(cam, R=T[:3, :3], t=T[:3, 3]), cfg, wts))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g["pose"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, g["pose"][k])


def test_paper_approx_pose_gradient_is_the_frozen_covariance_derivative():
    """The paper drops the Sigma' path from the pose gradient (Sec. 3.3 and
    the supplement): the approximate gradient is the derivative of the
    objective when every Gaussian's screen covariance stays at its base-pose
    value while its projected centre and depth follow the perturbed pose.
    FP64 central differences in smooth mode, with the covariance of the
    perturbed projections replaced by the base pose's."""
    sc, cam = _fd_scene(), _fd_cam()
    cfg = O.Config.smooth(bg=(0.3, 0.6, 0.9)).as_f32()
    wts = _weights(cam)
    ga = O.render_backward(sc, cam, cfg, *wts, approx_pose=True)
    ge = O.render_backward(sc, cam, cfg, *wts)
    base = O.project(sc, cam, cfg)
    T0 = np.block([[np.asarray(cam.R, float), np.asarray(cam.t, float)[:, None]], [np.zeros((1, 3)), np.ones((1, 1))]])
    h = 1e-6
    for k in range(6):
        vals = []
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[k] = sgn * h
            T = W.se3_exp(xi) @ T0
            c2 = dataclasses.replace(cam, R=T[:3, :3], t=T[:3, 3])
            p = dict(O.project(sc, c2, cfg))
            p["conic"], p["cov2"] = base["conic"], base["cov2"]
            r = O.render(sc, c2, cfg, proj=p)
            vals.append(float(np.sum(wts[0] * r["rgb"]) + np.sum(wts[1] * r["depth"]) + np.sum(wts[2] * r["T_final"])))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - ga["pose"][k]) <= 1e-6 * (1 + abs(fd)), (k, fd, ga["pose"][k])
    # The dropped path is not negligible on this scene: the exact gradient differs.
    assert np.abs(ge["pose"] - ga["pose"]).max() > 1e-3 * np.abs(ge["pose"]).max()
    # Only the pose changes: the Gaussian parameters' gradients are the exact ones.
    for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        np.testing.assert_array_equal(ga[name], ge[name])


def test_depth_alpha_derivative_matches_printed_formula():
    """Single pixel, three Gaussians: dD/dalpha_i from eq. grad_depth,
    d_i prod_{j<i}(1-a_j) - sum_{k>i} d_k a_k prod_{j<k, j!=i}(1-a_j),
    equals the oracle's opacity gradient divided by dalpha/do."""
    cam = _cam(16, 16, 40.0)
    sc = _scene([((0.01, 0.0, 1.5), (math.log(0.1),) * 3, (1, 0, 0, 0), 0.3, (0.1, 0.2, 0.3)),
                 ((0.0, 0.02, 2.5), (math.log(0.15),) * 3, (1, 0, 0, 0), -0.2, (0.4, 0.5, 0.6)),
                 ((-0.02, 0.0, 3.5), (math.log(0.2),) * 3, (1, 0, 0, 0), 0.7, (0.7, 0.8, 0.9))])
    cfg = O.Config().as_f32()
    px, py = 8, 7
    gD = np.zeros((16, 16))
    gD[py, px] = 1.0
    g = O.render_backward(sc, cam, cfg, np.zeros((3, 16, 16)), gD, None)
    p = g["fwd"]["proj"]
    order = np.argsort(p["z"])
    al, G = [], []
    for i in order:
        a_, b_, c_ = p["conic"][i]
        dx, dy = p["uv"][i, 0] - px, p["uv"][i, 1] - py
        Gi = math.exp(-0.5 * (a_ * dx * dx + 2 * b_ * dx * dy + c_ * dy * dy))
        G.append(Gi)
        al.append(p["opacity"][i] * Gi)
    d = p["z"][order]
    for ii, i in enumerate(order):
        first = d[ii] * np.prod([1 - al[j] for j in range(ii)])
        rest = sum(d[k] * al[k] * np.prod([1 - al[j] for j in range(k) if j != ii]) for k in range(ii + 1, 3))
        printed = first - rest
        ours = g["grad2d"][i, 5] / G[ii]
        assert abs(printed - ours) < 1e-12


def test_colour_gradients_sum_to_accumulated_opacity():
    sc = W.random_scene(500, seed=8)
    cam = W.camera_small()
    cfg = O.Config().as_f32()
    fwd = O.render(sc, cam, cfg)
    for (py, px) in [(60, 80), (10, 10), (100, 150)]:
        gC = np.zeros((3, cam.height, cam.width))
        gC[0, py, px] = 1.0
        g2, _ = O.backward_2d(sc, cam, cfg, gC, np.zeros((cam.height, cam.width)), None, fwd=fwd)
        assert abs(g2[:, 6].sum() - (1 - fwd["T_final"][py, px])) < 1e-12


def test_translation_gauge_identity():
    """dL/drho = R sum_i dL/dmu_i: moving the camera equals moving every mean.
    The identity holds with the exact pose gradient."""
    sc = W.random_scene(800, seed=12)
    cam = W.perturb_pose(W.camera_small(), [0.05, -0.02, 0.1, 0.02, 0.03, -0.01])
    gr, gd, gt = W.upstream_grads([(cam.width, cam.height)], seed=5)
    g = O.render_backward(sc, cam, O.Config(), gr.reshape(3, 120, 160), gd.reshape(120, 160), gt.reshape(120, 160))
    lhs = g["pose"][:3]
    rhs = np.asarray(cam.R, float) @ g["mean"].sum(0)
    # R is float32-rounded, so orthonormal only to ~1e-7.
    np.testing.assert_allclose(lhs, rhs, rtol=5e-7, atol=5e-7 * np.abs(lhs).max())
    ga = O.render_backward(sc, cam, O.Config(), gr.reshape(3, 120, 160), gd.reshape(120, 160),
                           gt.reshape(120, 160), approx_pose=True)
    assert np.abs(ga["pose"][:3] - lhs).max() > 1e-3 * np.abs(lhs).max()


def test_l1_loss_definition():
    rgb = np.array([[[0.5, 0.2], [0.1, 0.9]]] * 3)
    trgb = rgb.copy()
    trgb[0, 0, 0] = 0.7
    trgb[1, 1, 1] = 0.4
    depth = np.array([[1.0, 2.0], [3.0, 4.0]])
    tdep = np.array([[1.5, 0.0], [3.0, 3.0]])
    mask = np.array([[1, 1], [1, 0]], np.uint8)
    loss, gC, gD = O.l1_loss(rgb, depth, trgb, tdep, mask, w_rgb=0.8, w_depth=0.3)
    # brute-force sum
    ref = 0.0
    for y in range(2):
        for x in range(2):
            if not mask[y, x]:
                continue
            ref += 0.8 * sum(abs(rgb[c, y, x] - trgb[c, y, x]) for c in range(3))
            if tdep[y, x] > 0:
                ref += 0.3 * abs(depth[y, x] - tdep[y, x])
    assert abs(loss - ref) < 1e-12
    assert gC[0, 0, 0] == -0.8 and gC[1, 1, 1] == 0.0 and gC[2, 0, 0] == 0.0  # masked / sign(0) = 0
    assert gD[0, 0] == -0.3 and gD[0, 1] == 0.0 and gD[1, 0] == 0.0 and gD[1, 1] == 0.0


def test_reliable_selection_cases():
    """Eq. 12: keep a Gaussian whose centre depth agrees with the observed
    depth at its pixel; drop a floater in front of (or behind) the surface;
    keep Gaussians without evidence (outside the image, behind the near
    plane, missing reading); an excluded Gaussian stays excluded."""
    cam = _cam(32, 24, 30.0)
    depth = np.full((24, 32), 2.0, np.float32)
    depth[0:4, 0:4] = 0.0  # missing readings in the top-left corner
    rows = [((0.0, 0.0, 2.03), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),   # on the surface
            ((0.05, 0.0, 1.2), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),   # floater in front
            ((0.0, 0.05, 2.6), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),   # behind the surface
            ((5.0, 0.0, 2.0), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),    # outside the image
            ((0.0, 0.0, 0.1), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),    # before the near plane
            ((-0.98, -0.7, 1.0), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5)),  # missing reading
            ((0.0, 0.0, 2.0), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5))]    # excluded by the mask
    sc = _scene(rows)
    pix = O.project(sc, cam, O.Config())["uv"][5]
    assert np.all(np.floor(pix + 0.5) < 4)  # really lands in the missing corner
    got = O.select_reliable(sc, cam, depth, eps=0.1, mask=np.array([1, 1, 1, 1, 1, 1, 0]))
    assert list(got) == [1, 0, 0, 1, 1, 1, 0]
    # The decision is |D - z| <= eps, inclusive.
    sc2 = _scene([((0.0, 0.0, 2.0 + 0.0625), (-3, -3, -3), (1, 0, 0, 0), 0.0, (0.5, 0.5, 0.5))])
    assert list(O.select_reliable(sc2, cam, depth, eps=0.0625)) == [1]
    assert list(O.select_reliable(sc2, cam, depth, eps=0.0624)) == [0]


# ----------------------------------------------------------------- loss cap

def _rank_element(vals, k):
    """Brute force: the value x with #(v < x) <= k < #(v <= x) under the
    order of non-negative floats (negatives and -0 as 0, NaN last)."""
    def key(x):
        return (1, 0.0) if math.isnan(x) else (0, max(x, 0.0))
    for x in vals:
        below = sum(key(v) < key(x) for v in vals)
        upto = sum(key(v) <= key(x) for v in vals)
        if below <= k < upto:
            return key(x)
    raise AssertionError("no element of rank k")


def test_loss_median_is_the_lower_median_by_brute_force():
    rng = np.random.default_rng(4)
    for trial in range(60):
        m = int(rng.integers(1, 12))
        v = rng.choice([0.0, -0.0, 0.25, 0.5, 1.0, 3.0, -2.0, np.inf, np.nan], size=m) if trial % 2 else \
            rng.random(m).astype(np.float32)
        v = np.asarray(v, np.float32)
        got = O.loss_median(v)
        want = _rank_element(v.tolist(), (m - 1) // 2)
        if want[0] == 1:
            assert np.isnan(got)
        else:
            assert float(got) == want[1], (v, got, want)
    # odd counts of distinct positive values: numpy's median
    v = np.random.default_rng(5).random(101).astype(np.float32)
    assert O.loss_median(v) == np.float32(np.median(v))
    # even count: the lower of the two middle values
    assert O.loss_median(np.array([4.0, 1.0, 3.0, 2.0], np.float32)) == np.float32(2.0)
    # mask, and no eligible pixel
    mask = np.array([0, 1, 1, 0], np.uint8)
    assert O.loss_median(np.array([9.0, 1.0, 5.0, 0.0], np.float32), mask) == np.float32(1.0)
    assert O.loss_median(np.zeros(3, np.float32), np.zeros(3, np.uint8)) is None
    assert O.loss_cap(np.zeros(3, np.float32), np.zeros(3, np.uint8)) == np.inf
    assert O.loss_cap(np.array([1.5, 0.5, 2.5], np.float32), None, 10.0) == np.float32(15.0)


def test_l1_loss_cap_drops_pixels_above_it():
    rng = np.random.default_rng(6)
    H, Wd = 5, 7
    rgb, trgb = rng.random((3, H, Wd)), rng.random((3, H, Wd))
    dep, tdep = rng.random((H, Wd)) + 1, rng.random((H, Wd)) + 1
    tdep[0, :3] = 0.0
    w_rgb, w_d = 0.8, 0.3
    # each pixel's own term, written out pixel by pixel
    lp = np.zeros((H, Wd))
    for y in range(H):
        for x in range(Wd):
            lp[y, x] = w_rgb * sum(abs(rgb[c, y, x] - trgb[c, y, x]) for c in range(3))
            if tdep[y, x] > 0:
                lp[y, x] += w_d * abs(dep[y, x] - tdep[y, x])
    np.testing.assert_allclose(O.l1_pixel_loss(rgb, dep, trgb, tdep, None, w_rgb, w_d), lp, rtol=1e-14)
    cap = float(np.median(lp))
    L, gC, gD = O.l1_loss(rgb, dep, trgb, tdep, None, w_rgb, w_d, loss_cap=cap)
    keep = lp <= cap
    assert abs(L - lp[keep].sum()) <= 1e-12 * lp.sum()
    assert not gC[:, ~keep].any() and not gD[~keep].any()
    L0, gC0, gD0 = O.l1_loss(rgb, dep, trgb, tdep, None, w_rgb, w_d)
    np.testing.assert_array_equal(gC[:, keep], gC0[:, keep])
    Linf, _, _ = O.l1_loss(rgb, dep, trgb, tdep, None, w_rgb, w_d, loss_cap=np.inf)
    assert Linf == L0
