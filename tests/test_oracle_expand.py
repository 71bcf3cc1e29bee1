"""Pins of the oracle's map expansion (Sec. 3.2: adding step Eq. 8,
deleting step Eq. 9) against brute force, geometric identities and
hand-built cases -- none of which re-types the oracle's own formulas."""
import math

import numpy as np
import pytest

import oracle.expand as E
import workloads as W


def _posed(cam, seed):
    rng = np.random.default_rng(seed)
    xi = np.concatenate([rng.normal(0, 0.3, 3), rng.normal(0, 0.2, 3)])
    return W.perturb_pose(cam, xi)


def test_adding_mask_brute_force():
    """Pixel by pixel with Python floats: a reading and (1 - T < tau_T or
    |D - D_hat| > tau_D); thresholds planted exactly (strict comparisons, so
    those pixels stay reliable unless the other test fires), zero and NaN
    readings never added."""
    tau_T, tau_D = 0.5, 0.25
    T, dr, do, _ = W.expansion_images([(23, 17)], seed=2, plant_tau_T=tau_T, plant_tau_D=tau_D)
    m = E.adding_mask(T, dr, do, tau_T, tau_D)
    n_plant_T = n_plant_D = 0
    for k in range(T.size):
        t, d_hat, d = float(T[k]), float(dr[k]), float(do[k])
        want = False
        if d > 0.0:
            a = 1.0 - t
            want = (a < tau_T) or (abs(d - d_hat) > tau_D)
        assert bool(m[k]) == want, k
        n_plant_T += t == 0.5
        n_plant_D += (d_hat == 1.0 and d == 1.25)
    assert n_plant_T > 0 and n_plant_D > 0
    # an exactly planted depth error alone does not add the pixel
    sel = (dr == 1.0) & (do == 1.25) & (T < 0.5)
    assert sel.any() and not m[sel].any()
    assert not m[~(do > 0)].any() and m.any() and not m.all()


def test_back_projection_round_trip():
    """Projecting the back-projected point with the pinhole camera gives the
    pixel back and the camera-frame depth D (to 1e-6: the float32 rotation is
    orthonormal only to float32 rounding, so its transpose inverts it to
    ~1e-7)."""
    cam = _posed(W.camera_small(), 3)
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, y = rng.integers(0, cam.width), rng.integers(0, cam.height)
        D = rng.uniform(0.3, 6.0)
        X = E.back_project(int(x), int(y), D, cam)
        Xc = R @ X + t
        assert Xc[2] == pytest.approx(D, rel=1e-6)
        assert cam.fx * Xc[0] / Xc[2] + cam.cx == pytest.approx(x, abs=1e-4)
        assert cam.fy * Xc[1] / Xc[2] + cam.cy == pytest.approx(y, abs=1e-4)
    # with an exactly orthonormal rotation the round trip is exact to FP64
    cam2 = W.camera_small().with_pose(np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]), [0.25, -0.5, 1.0])
    X = E.back_project(17, 93, 2.5, cam2)
    Xc = np.asarray(cam2.R, np.float64) @ X + np.asarray(cam2.t, np.float64)
    np.testing.assert_allclose(Xc, 2.5 * np.array([(17 - cam2.cx) / cam2.fx, (93 - cam2.cy) / cam2.fy, 1.0]),
                               rtol=1e-14, atol=1e-14)


def test_new_scale_is_the_spacing_of_neighbouring_pixels():
    """On a fronto-parallel surface at depth D the back-projections of
    horizontally and vertically adjacent pixels lie D/fx and D/fy apart; the
    new isotropic scale is their geometric mean (times the factor)."""
    cam = W.camera_small().with_size(150.0, 120.0, 79.5, 59.5, 160, 120)
    D = 2.5
    a, b, c = (E.back_project(x, y, D, cam) for x, y in ((40, 30), (41, 30), (40, 31)))
    dx, dy = np.linalg.norm(b - a), np.linalg.norm(c - a)
    assert dx == pytest.approx(D / 150.0, rel=1e-12) and dy == pytest.approx(D / 120.0, rel=1e-12)
    sizes = [(cam.width, cam.height)]
    T = np.zeros(cam.width * cam.height, np.float32)  # every pixel has opacity 1: reliable...
    dr = np.full_like(T, D)
    do = np.full_like(T, D)
    do[5] = D + 1.0  # ...except this one (depth error 1 m)
    _, new = E.add_gaussians([cam], [T.reshape(120, 160)], [dr.reshape(120, 160)], [do.reshape(120, 160)],
                             [np.zeros((3, 120, 160), np.float32)], 0.1, 0.5, 1.5, 0.0)
    assert new["mean"].shape == (1, 3)
    s = math.exp(new["log_scale"][0, 0])
    assert s == pytest.approx(1.5 * (D + 1.0) / math.sqrt(150.0 * 120.0), rel=1e-12)
    assert tuple(new["pixel"][0]) == (0, 5, 0)
    del sizes


def test_add_gaussians_order_colour_and_initialisation():
    """Two ragged posed views: one new Gaussian per unreliable pixel, in view
    then row-major order, at a point on the pixel's ray at the observed
    depth, with the observed colour, identity rotation and the initial
    opacity."""
    sizes = [(37, 21), (16, 33)]
    cams = [_posed(W.camera_small().with_size(40.0, 44.0, 18.0, 10.0, 37, 21), 5),
            _posed(W.camera_small().with_size(30.0, 30.0, 7.5, 16.0, 16, 33), 6)]
    T, dr, do, rgb = W.expansion_images(sizes, seed=7)
    parts, po = [], 0
    for w, h in sizes:
        n = w * h
        parts.append((T[po:po + n].reshape(h, w), dr[po:po + n].reshape(h, w), do[po:po + n].reshape(h, w),
                      rgb[3 * po:3 * po + 3 * n].reshape(3, h, w)))
        po += n
    masks, new = E.add_gaussians(cams, *[list(x) for x in zip(*parts)], 0.3, 0.15, 1.0, -2.0)
    assert len(new["mean"]) == sum(int(m.sum()) for m in masks) > 0
    keys = [tuple(p) for p in new["pixel"]]
    assert keys == sorted(keys, key=lambda k: (k[0], k[2], k[1]))
    for j, (v, x, y) in enumerate(keys):
        assert masks[v][y, x]
        cam = cams[v]
        Xc = np.asarray(cam.R, np.float64) @ new["mean"][j] + np.asarray(cam.t, np.float64)
        D = float(parts[v][2][y, x])
        ray = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
        np.testing.assert_allclose(Xc, D * ray, rtol=1e-6, atol=1e-7)
        np.testing.assert_array_equal(new["rgb"][j], parts[v][3][:, y, x].astype(np.float64))
    np.testing.assert_array_equal(new["quat"], np.tile([1.0, 0.0, 0.0, 0.0], (len(keys), 1)))
    assert (new["opacity_logit"] == -2.0).all()


def _plane_cam():
    cam = W.camera_small().with_size(100.0, 100.0, 50.0, 40.0, 101, 81)
    return cam.with_pose(np.eye(3), np.zeros(3))


def test_delete_hand_built_cases():
    """A fronto-parallel surface 3 m in front of an identity camera
    (gamma 0.5 m, eta 0.01): on-axis Gaussians at 1 m (2 m in front: decayed,
    opacity times eta exactly) and at 2.8 m (0.2 m: kept); behind the surface,
    off the image, before the near plane, on a pixel without a reading, or
    masked out: kept.  An off-axis one at (1, 0, 1): its ray meets the surface
    at (3, 0, 3), 2 sqrt(2) m beyond it -> decayed."""
    cam = _plane_cam()
    depth = np.full((81, 101), 3.0, np.float32)
    depth[40, 60] = 0.0  # no reading where (0.2, 0, 2) projects
    mean = np.array([[0, 0, 1.0], [0, 0, 2.8], [0, 0, 4.0], [10.0, 0, 1.0], [0, 0, 0.1], [0.2, 0, 2.0],
                     [0, 0, 1.5], [0.5, 0, 1.0]], np.float32)
    logit = np.array([0.3, 0.3, 0.3, 0.3, 0.3, 0.3, 0.3, -1.0], np.float32)
    mask = np.array([1, 1, 1, 1, 1, 1, 0, 1], np.uint8)
    out, dec = E.delete_gaussians(mean, logit, cam, depth, gamma=0.5, eta=0.01, mask=mask)
    assert dec.tolist() == [True, False, False, False, False, False, False, True]
    sig = lambda v: 1.0 / (1.0 + math.exp(-v))  # noqa: E731
    assert sig(out[0]) == pytest.approx(float(np.float32(0.01)) * sig(float(np.float32(0.3))), rel=1e-12)
    assert sig(out[7]) == pytest.approx(float(np.float32(0.01)) * sig(-1.0), rel=1e-12)
    assert (out[1:7] == np.float32(0.3)).all()
    # (1, 0, 1) projects to u = 150: outside; (0.5, 0, 1) at u = 100 inside
    # the 101-wide image: surface point (1.5, 0, 3), distance sqrt(1 + 4);
    # gamma a float32 step either side of it (gamma is taken as float32).
    dist = math.dist((0.5, 0, 1.0), (1.5, 0, 3.0))
    _, dec2 = E.delete_gaussians(mean[7:], logit[7:], cam, depth, gamma=dist - 1e-5, eta=0.5)
    _, dec3 = E.delete_gaussians(mean[7:], logit[7:], cam, depth, gamma=dist + 1e-5, eta=0.5)
    assert dec2[0] and not dec3[0]


def test_delete_matches_world_space_distance():
    """Random scene and posed camera: the decision equals the printed
    condition written with world points -- P_uv the back-projection of the
    ray's image point (u, v) at the observed depth (through the camera's
    extrinsics), dist the Euclidean distance to X_i, counted positive when the
    surface lies beyond the Gaussian -- on every Gaussian not within 1e-9 of
    gamma."""
    cam = _posed(W.camera_small(), 9)
    sc = W.random_scene(600, seed=4, z=(0.5, 6.0))
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    Xc_all = sc.mean.astype(np.float64) @ R.T + t
    rng = np.random.default_rng(1)
    depth = rng.uniform(1.0, 7.0, size=(cam.height, cam.width)).astype(np.float32)
    depth[rng.random(depth.shape) < 0.1] = 0.0
    gamma = 0.3
    _, dec = E.delete_gaussians(sc.mean, sc.opacity_logit, cam, depth, gamma=gamma, eta=0.1)
    checked = fired = 0
    for i in range(sc.n):
        Xc = Xc_all[i]
        want = False
        if Xc[2] > 0.2:
            u = cam.fx * Xc[0] / Xc[2] + cam.cx
            v = cam.fy * Xc[1] / Xc[2] + cam.cy
            px, py = math.floor(u + 0.5), math.floor(v + 0.5)
            if 0 <= px < cam.width and 0 <= py < cam.height and depth[py, px] > 0:
                D = float(depth[py, px])
                P_uv = E.back_project(u, v, D, cam)
                d = float(np.linalg.norm(sc.mean[i].astype(np.float64) - P_uv))
                signed = d if D > Xc[2] else -d
                if abs(signed - gamma) < 1e-9:
                    continue
                want = signed > gamma
        checked += 1
        fired += want
        assert bool(dec[i]) == want, i
    assert checked > 500 and 20 < fired < checked - 20


def test_new_gaussian_in_a_spherical_harmonic_map_renders_its_observed_colour():
    """A new Gaussian of a spherical-harmonic map (degree 1) rendered alone,
    from two cameras seeing it along different directions, gives the image
    of the same Gaussian in the RGB model with the observed colour: its
    coefficients carry the colour in the constant term only."""
    import oracle as O
    sizes = [(37, 21)]
    cams = [_posed(W.camera_small().with_size(40.0, 44.0, 18.0, 10.0, 37, 21), 5)]
    T, dr, do, rgb = W.expansion_images(sizes, seed=7)
    w, h = sizes[0]
    masks, new = E.add_gaussians(cams, [T.reshape(h, w)], [dr.reshape(h, w)], [do.reshape(h, w)],
                                 [rgb.reshape(3, h, w)], 0.3, 0.15, 1.0, 1.5)
    assert len(new["mean"]) >= 3
    for j in range(3):
        mean = new["mean"][j:j + 1].astype(np.float32)
        ls = np.full((1, 3), math.log(0.05), np.float32)
        base = dict(mean=mean, log_scale=ls, quat=new["quat"][j:j + 1].astype(np.float32),
                    opacity_logit=new["opacity_logit"][j:j + 1].astype(np.float32))
        rgb_scene = W.Scene(rgb=new["rgb"][j:j + 1].astype(np.float32), **base)
        sh_scene = W.Scene(rgb=np.zeros((1, 3), np.float32), sh=new["sh"][j:j + 1].astype(np.float32), **base)
        for k, xi in enumerate(([0.0] * 6, [0.08, -0.05, 0.02, 0.1, -0.15, 0.05])):
            # A camera looking at the Gaussian from 1.5 m, then moved by xi.
            c = W.camera_small().with_size(60.0, 60.0, 31.5, 23.5, 64, 48)
            R0 = np.eye(3)
            t0 = -(R0 @ mean[0].astype(np.float64)) + np.array([0.0, 0.0, 1.5])
            cam = W.perturb_pose(c.with_pose(R0, t0), xi)
            a = O.render(rgb_scene, cam, O.Config())
            b = O.render(sh_scene, cam, O.Config())
            assert a["rgb"].max() > 0.01, (j, k)
            np.testing.assert_allclose(b["rgb"], a["rgb"], rtol=0, atol=1e-6)
