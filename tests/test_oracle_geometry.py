"""Pins of the oracle's geometry (Eq. 2, Eq. 3, eq. q2R, eq. grad_q, eq. grad_m)
against closed forms, library routines and brute force -- never against the
oracle's own formulas retyped."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.golden.load import evaluate, load_expressions

RNG = np.random.default_rng(1234)


def _hamilton(p, q):
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_q2R_matches_quaternion_conjugation():
    q = RNG.normal(size=(50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = O.quat_to_rotmat(q)
    for k in range(50):
        v = RNG.normal(size=3)
        qv = _hamilton(_hamilton(q[k], np.r_[0.0, v]), q[k] * np.array([1, -1, -1, -1]))
        np.testing.assert_allclose(R[k] @ v, qv[1:], atol=1e-12)
        np.testing.assert_allclose(R[k].T @ R[k], np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R[k]) - 1.0) < 1e-12


def test_q2R_special_case_quarter_turn_about_z():
    c = math.sqrt(0.5)
    R = O.quat_to_rotmat(np.array([[c, 0.0, 0.0, c]]))[0]
    np.testing.assert_allclose(R, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-15)


def test_dR_dq_matches_printed_closed_form():
    """The derivative matrices of eq. grad_q (one sign corrected) applied to
    a point equal the oracle's dR/dq applied to the same point."""
    table = load_expressions("dXc_dq.txt")
    q = RNG.normal(size=(20, 4))
    grads = O.quat_to_rotmat_grads(q)
    for k in range(20):
        p = RNG.normal(size=3)
        env = dict(qr=q[k, 0], qi=q[k, 1], qj=q[k, 2], qk=q[k, 3], x=p[0], y=p[1], z=p[2])
        for name, dR in zip(("q_r", "q_i", "q_j", "q_k"), grads):
            rows = np.array(evaluate(table[name], env), dtype=float)
            printed = 2.0 * rows.sum(axis=1)
            np.testing.assert_allclose(dR[k] @ p, printed, atol=1e-12)


def test_dR_dq_matches_finite_differences():
    q = RNG.normal(size=(10, 4))
    grads = O.quat_to_rotmat_grads(q)
    h = 1e-6
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        fd = (O.quat_to_rotmat(q + e) - O.quat_to_rotmat(q - e)) / (2 * h)
        np.testing.assert_allclose(grads[j], fd, atol=1e-8)


def test_covariance_eigen_decomposition():
    sc = W.random_scene(40, seed=3)
    Sigma, R, s, _, _ = O.covariance_3d(sc.log_scale.astype(float), sc.quat.astype(float))
    for k in range(40):
        evals, evecs = np.linalg.eigh(Sigma[k])
        np.testing.assert_allclose(evals, np.sort(s[k] ** 2), rtol=1e-10)
        # each column of R is an eigenvector with eigenvalue s_j^2
        for j in range(3):
            np.testing.assert_allclose(Sigma[k] @ R[k][:, j], s[k, j] ** 2 * R[k][:, j], atol=1e-14)


def _one_gaussian(mean, log_scale, quat=(1, 0, 0, 0), op=0.0, rgb=(0.2, 0.4, 0.6)):
    return W.Scene(np.array([mean], np.float64), np.array([log_scale], np.float64),
                   np.array([quat], np.float64), np.array([op], np.float64), np.array([rgb], np.float64))


def test_ewa_closed_form_isotropic_on_axis():
    cam = W.camera_small()
    s, z = 0.05, 2.0
    sc = _one_gaussian([0, 0, z], [math.log(s)] * 3, quat=(0.3, -0.5, 0.1, 0.8))
    cfg = O.Config().as_f32()
    p = O.project(sc, cam, cfg)
    sig = (cam.fx * s / z) ** 2 + cfg.lowpass
    np.testing.assert_allclose(p["cov2"][0], [[sig, 0], [0, sig]], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(p["uv"][0], [cam.cx, cam.cy], atol=1e-12)
    np.testing.assert_allclose(p["conic"][0], [1 / sig, 0, 1 / sig], rtol=1e-12)


def test_jacobian_matches_numerical_projection_derivative():
    cam = W.camera_small()
    sc = W.random_scene(8, seed=5)
    p = O.project(sc, cam, O.Config(fov_guard=0.0))  # Eq. 3 as printed

    def proj(X):
        return np.array([cam.fx * X[0] / X[2] + cam.cx, cam.fy * X[1] / X[2] + cam.cy])

    h = 1e-6
    for k in range(8):
        X = p["Xc"][k]
        Jn = np.stack([(proj(X + h * e) - proj(X - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(p["J"][k], Jn, rtol=1e-7, atol=1e-6)


def test_guarded_jacobian_is_projection_derivative_at_the_limit():
    """With the guard on, J is the derivative of the pinhole projection at
    the point whose x/z and y/z are clipped to +-g W/(2 fx), +-g H/(2 fy);
    the projected centre is unchanged."""
    cam = W.camera_small()
    sc = W.random_scene(40, seed=5, xy=2.5)
    g = 1.3
    p = O.project(sc, cam, O.Config(fov_guard=g))
    p0 = O.project(sc, cam, O.Config(fov_guard=0.0))
    lx, ly = g * cam.width / (2 * cam.fx), g * cam.height / (2 * cam.fy)

    def proj(X):
        return np.array([cam.fx * X[0] / X[2] + cam.cx, cam.fy * X[1] / X[2] + cam.cy])

    h = 1e-6
    n_clip = 0
    for k in range(sc.n):
        x, y, z = p["Xc"][k]
        Xl = np.array([np.clip(x / z, -lx, lx) * z, np.clip(y / z, -ly, ly) * z, z])
        n_clip += int(abs(x / z) > lx or abs(y / z) > ly)
        Jn = np.stack([(proj(Xl + h * e) - proj(Xl - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(p["J"][k], Jn, rtol=1e-7, atol=1e-6)
    assert 5 <= n_clip <= sc.n - 5, n_clip
    np.testing.assert_array_equal(p["uv"], p0["uv"])


def test_ewa_covariance_matches_sampled_projection():
    """For a small Gaussian the linearised projection is exact: the covariance
    of projected samples equals Sigma' minus the low-pass term."""
    cam = W.camera_small()
    rng = np.random.default_rng(7)
    sc = _one_gaussian([0.3, -0.2, 2.5], [math.log(0.004), math.log(0.002), math.log(0.003)],
                       quat=(0.7, 0.2, -0.4, 0.3))
    cam = cam.with_pose(W.se3_exp([0.1, 0.0, 0.2, 0.05, -0.1, 0.2])[:3, :3],
                        W.se3_exp([0.1, 0.0, 0.2, 0.05, -0.1, 0.2])[:3, 3])
    cfg = O.Config().as_f32()
    p = O.project(sc, cam, cfg)
    L = np.linalg.cholesky(p["Sigma"][0])
    X = sc.mean[0] + rng.normal(size=(400_000, 3)) @ L.T
    Xc = X @ np.asarray(cam.R, float).T + np.asarray(cam.t, float)
    uv = np.stack([cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx, cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy], 1)
    emp = np.cov(uv.T)
    expect = p["cov2"][0] - cfg.lowpass * np.eye(2)
    np.testing.assert_allclose(emp, expect, rtol=2e-2, atol=2e-2 * np.abs(expect).max())


def test_sigma2d_backward_matches_printed_dvec_dE():
    """With an identity camera rotation E = J, and the printed derivative of
    vec(Sigma') w.r.t. each e_kl contracted with dL/dSigma' must equal the
    oracle's dL/dJ."""
    table = load_expressions("dvecSigma2d_dE.txt")
    for _ in range(10):
        J = RNG.normal(size=(1, 2, 3))
        A = RNG.normal(size=(3, 3))
        S = (A @ A.T)[None]
        G = RNG.normal(size=(2, 2))
        G = (G + G.T)[None]
        _, GJ = O.sigma2d_backward(G, J, S)
        env = {f"e{i}{j}": J[0, i, j] for i in range(2) for j in range(3)}
        env.update({f"S{i}{j}": S[0, i, j] for i in range(3) for j in range(3)})
        gvec = G[0].reshape(4)
        for i in range(2):
            for j in range(3):
                d = np.array(evaluate(table[f"e{i}{j}"], env), dtype=float)
                assert abs(gvec @ d - GJ[0, i, j]) < 1e-10 * (1 + abs(GJ[0, i, j]))


def test_rect_half_width_is_ellipse_extent():
    """Brute force: the 3-sigma ellipse boundary sampled densely reaches exactly
    the rectangle half-widths k*sqrt(Sigma'_00), k*sqrt(Sigma'_11)."""
    cam = W.camera_small()
    sc = W.random_scene(20, seed=9)
    cfg = O.Config().as_f32()
    p = O.project(sc, cam, cfg)
    th = np.linspace(0, 2 * np.pi, 200_001)
    circ = np.stack([np.cos(th), np.sin(th)])
    for k in np.nonzero(p["valid"])[0]:
        L = np.linalg.cholesky(p["cov2"][k])
        pts = cfg.cutoff * (L @ circ)
        rx = cfg.cutoff * math.sqrt(p["cov2"][k][0, 0])
        ry = cfg.cutoff * math.sqrt(p["cov2"][k][1, 1])
        assert abs(pts[0].max() - rx) <= 1e-8 * rx
        assert abs(pts[1].max() - ry) <= 1e-8 * ry


def test_culling_rules():
    cam = W.camera_small()
    cfg = O.Config()
    sc = _one_gaussian([0, 0, 0.1], [-3, -3, -3])  # in front of the camera but closer than z_near
    assert not O.project(sc, cam, cfg)["valid"][0]
    sc = _one_gaussian([0, 0, -2.0], [-3, -3, -3])  # behind
    assert not O.project(sc, cam, cfg)["valid"][0]
    sc = _one_gaussian([50.0, 0, 2.0], [-3, -3, -3])  # far outside the image
    assert not O.project(sc, cam, cfg)["valid"][0]
    sc = _one_gaussian([0, 0, 2.0], [-3, -3, np.nan])  # non-finite
    assert not O.project(sc, cam, cfg)["valid"][0]
    sc = _one_gaussian([0, 0, 2.0], [-3, -3, -3], quat=(0, 0, 0, 0))  # zero quaternion
    assert not O.project(sc, cam, cfg)["valid"][0]
    sc = _one_gaussian([0, 0, 2.0], [-3, -3, -3])
    assert O.project(sc, cam, cfg)["valid"][0]


@pytest.mark.parametrize("seed,n,size", [(0, 300, (53, 37)), (1, 500, (64, 48)), (2, 200, (17, 80))])
def test_tile_lists_match_brute_force(seed, n, size):
    """Brute force: each tile scans all Gaussians for the ones whose
    rectangle holds it and orders them with Python's sorted() on (float32
    depth bits, index)."""
    cam = W.camera_small().with_size(60.0, 60.0, (size[0] - 1) / 2, (size[1] - 1) / 2, *size)
    sc = W.random_scene(n, seed=seed)
    sc.mean[: n // 10, 2] = sc.mean[n // 10: 2 * (n // 10), 2]  # force equal depths (index tie-break)
    cfg = O.Config().as_f32()
    p = O.project(sc, cam, cfg)
    starts, gauss = O.tile_lists(p)
    ties = 0
    for tile in range(p["TX"] * p["TY"]):
        ty, tx = divmod(tile, p["TX"])
        members = []
        for i in range(n):
            if not p["valid"][i]:
                continue
            tx0, tx1, ty0, ty1 = p["rect"][i]
            if tx0 <= tx <= tx1 and ty0 <= ty <= ty1:
                members.append((int(np.float32(p["z"][i]).view(np.uint32)), i))
        ties += len(members) - len({m[0] for m in members})
        expect = [i for _, i in sorted(members)]
        assert list(gauss[starts[tile]:starts[tile + 1]]) == expect
    assert ties > 0
    assert not p["bin_ambiguous"].any()


def test_tile_alpha_max_closed_forms():
    """Largest alpha of a Gaussian over a tile's pixel centres: an isotropic
    Gaussian centred on a pixel centre of the tile reaches min(alpha_max, o)
    there; centred off the tile, its nearest pixel centre (the centre
    clamped to the tile's pixel range) gives o exp(-d^2 / (2 s^2)); a tile
    cut by the image edge only counts its pixels inside the image."""
    s2 = 9.0
    p = dict(TX=4, uv=np.array([[21.0, 5.0], [40.5, 7.25], [10.0, 20.0]]),
             conic=np.array([[1 / s2, 0.0, 1 / s2]] * 3), opacity=np.array([0.995, 0.6, 0.7]))
    cfg = O.Config().as_f32()
    got = O.tile_alpha_max(p, 1, [0, 1, 2], 64, 30, cfg)   # tile (tx 1, ty 0): x 16..31, y 0..15
    want = [min(cfg.alpha_max, 0.995),
            0.6 * math.exp(-((40.5 - 31) ** 2 + 0.25 ** 2) / (2 * s2)),
            0.7 * math.exp(-((16 - 10.0) ** 2 + (20 - 15) ** 2) / (2 * s2))]
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # tile (tx 0, ty 1) of a 64x18 image holds rows 16 and 17 only
    got = O.tile_alpha_max(p, 4, [2], 64, 18, cfg)
    np.testing.assert_allclose(got, [0.7 * math.exp(-(3 ** 2) / (2 * s2))], rtol=1e-12)
    assert O.tile_alpha_max(p, 4, [], 64, 18, cfg).size == 0


def test_rect_contains_every_pixel_inside_the_ellipse():
    """Every pixel with Q <= k^2 lies in a tile of the Gaussian's rectangle."""
    cam = W.camera_small()
    sc = W.random_scene(100, seed=11)
    cfg = O.Config().as_f32()
    p = O.project(sc, cam, cfg)
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    for k in np.nonzero(p["valid"])[0]:
        a, b, c = p["conic"][k]
        dx = p["uv"][k, 0] - px
        dy = p["uv"][k, 1] - py
        inside = a * dx * dx + 2 * b * dx * dy + c * dy * dy <= cfg.cutoff ** 2
        tx0, tx1, ty0, ty1 = p["rect"][k]
        tiles_x, tiles_y = px[inside] // 16, py[inside] // 16
        assert np.all((tiles_x >= tx0) & (tiles_x <= tx1) & (tiles_y >= ty0) & (tiles_y <= ty1))
