"""Seeded scene, camera and target generators (NumPy PCG64, fixed draw order).

Conventions shared by every consumer:
  * Gaussian parameters are float32 arrays: mean [N,3], log_scale [N,3],
    quat [N,4] stored (w, x, y, z), opacity_logit [N], rgb [N,3].
  * A camera holds pinhole intrinsics in pixels (pixel (x, y) has its centre
    at integer coordinates), a world->camera rotation R (3x3, row-major,
    float32) and translation t (3, float32) so that X_cam = R X + t, and the
    image size.  Camera axes: x right, y down, z forward.
  * The indoor "room box" spans x in [-3, 3], y in [-1.5, 1.5] (y points down,
    the floor is y = +1.5) and z in [-0.5, 3.5] metres.

Nothing here evaluates the renderer; poses are built with a plain SE(3)
exponential because perturbed and look-at cameras are inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # [3,3] float32, world -> camera
    t: np.ndarray  # [3] float32
    width: int
    height: int

    def __post_init__(self):
        # The renderer takes the intrinsics as float32: hold exactly those
        # values, so that the renderer and the oracle see the same camera
        # (poses from with_pose are float32 too).
        for k in ("fx", "fy", "cx", "cy"):
            setattr(self, k, float(np.float32(getattr(self, k))))

    def with_pose(self, R, t) -> "Camera":
        return dataclasses.replace(self, R=np.asarray(R, F32).reshape(3, 3).copy(),
                                   t=np.asarray(t, F32).reshape(3).copy())

    def with_size(self, fx, fy, cx, cy, width, height) -> "Camera":
        return dataclasses.replace(self, fx=fx, fy=fy, cx=cx, cy=cy,
                                   width=int(width), height=int(height))


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    rgb: np.ndarray
    # Optional degree-1 spherical-harmonic colour coefficients [N, 4, 3]
    # (coefficient k = 0..3, channel): when present, colour is view-dependent
    # and `rgb` is not used.
    sh: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def arrays(self):
        return (self.mean, self.log_scale, self.quat, self.opacity_logit, self.rgb)


def _identity_pose():
    return np.eye(3, dtype=F32), np.zeros(3, F32)


def _draw_appearance(rng, n, log_scale_mu=-3.0, log_scale_sd=0.5):
    """Log-scales N(mu, sd^2) per axis, uniform random unit quaternions,
    opacity logits N(0, 1), RGB uniform in [0, 1]^3 (in that draw order)."""
    log_scale = rng.normal(log_scale_mu, log_scale_sd, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, size=n)
    rgb = rng.random(size=(n, 3))
    return log_scale.astype(F32), q.astype(F32), opacity_logit.astype(F32), rgb.astype(F32)


def random_scene(n=2000, seed=0, xy=1.0, z=(1.0, 5.0), log_scale_mu=-3.0, log_scale_sd=0.5) -> Scene:
    """Means uniform in x, y in [-xy, xy], z in [z0, z1]; other parameters as
    _draw_appearance.  With the defaults this is the small forward workload
    (2 000 Gaussians in front of an identity camera)."""
    rng = np.random.default_rng(seed)
    mx = rng.uniform(-xy, xy, size=n)
    my = rng.uniform(-xy, xy, size=n)
    mz = rng.uniform(z[0], z[1], size=n)
    mean = np.stack([mx, my, mz], axis=1).astype(F32)
    ls, q, op, rgb = _draw_appearance(rng, n, log_scale_mu, log_scale_sd)
    return Scene(mean, ls, q, op, rgb)


def needle_scene(n=600, seed=0, z=(2.5, 3.5), half_width=1.0, sigma_y=(0.2, 0.5), sigma_thin=0.002) -> Scene:
    """Tall thin Gaussians in front of an identity camera: means uniform in
    x in [-half_width, half_width], y in [-0.2, 0.2], z in `z`; axis-aligned
    (identity quaternions) with scales (sigma_thin, U[sigma_y], sigma_thin)
    metres, so each covers many tile rows but one or two tile columns;
    opacity logits N(1, 1), RGB uniform in [0, 1]^3."""
    rng = np.random.default_rng(seed)
    mx = rng.uniform(-half_width, half_width, size=n)
    my = rng.uniform(-0.2, 0.2, size=n)
    mz = rng.uniform(z[0], z[1], size=n)
    sy = rng.uniform(sigma_y[0], sigma_y[1], size=n)
    log_scale = np.log(np.stack([np.full(n, sigma_thin), sy, np.full(n, sigma_thin)], axis=1))
    q = np.zeros((n, 4))
    q[:, 0] = 1.0
    opacity_logit = rng.normal(1.0, 1.0, size=n)
    rgb = rng.random(size=(n, 3))
    return Scene(np.stack([mx, my, mz], axis=1).astype(F32), log_scale.astype(F32), q.astype(F32),
                 opacity_logit.astype(F32), rgb.astype(F32))


# Room surfaces: (name, fixed axis, fixed value, outward-normal sign, area m^2).
_ROOM = dict(x=(-3.0, 3.0), y=(-1.5, 1.5), z=(-0.5, 3.5))
_SURFACES = (
    ("floor", 1, 1.5),   # 6 x 4 = 24 m^2
    ("back", 2, 3.5),    # 6 x 3 = 18 m^2
    ("front", 2, -0.5),  # 18 m^2
    ("left", 0, -3.0),   # 3 x 4 = 12 m^2
    ("right", 0, 3.0),   # 12 m^2
)
_AREAS = np.array([24.0, 18.0, 18.0, 12.0, 12.0])


def _surface_points(rng, n, offset_sd=0.01):
    lo = np.array([_ROOM["x"][0], _ROOM["y"][0], _ROOM["z"][0]])
    hi = np.array([_ROOM["x"][1], _ROOM["y"][1], _ROOM["z"][1]])
    which = rng.choice(len(_SURFACES), size=n, p=_AREAS / _AREAS.sum())
    uv = rng.random(size=(n, 3))
    pts = lo + uv * (hi - lo)
    off = rng.normal(0.0, offset_sd, size=n)
    for k, (_, axis, value) in enumerate(_SURFACES):
        sel = which == k
        pts[sel, axis] = value + off[sel]
    return pts


def room_scene(n=300_000, seed=0, surface_fraction=0.7) -> Scene:
    """Replica/TUM-shaped indoor scene: `surface_fraction` of the means lie on
    the floor and four walls (chosen by area, 1 cm normal jitter), the rest are
    uniform in the room box.  Appearance as _draw_appearance."""
    rng = np.random.default_rng(seed)
    n_surf = int(round(surface_fraction * n))
    surf = _surface_points(rng, n_surf)
    lo = np.array([_ROOM["x"][0], _ROOM["y"][0], _ROOM["z"][0]])
    hi = np.array([_ROOM["x"][1], _ROOM["y"][1], _ROOM["z"][1]])
    box = lo + rng.random(size=(n - n_surf, 3)) * (hi - lo)
    mean = np.concatenate([surf, box], axis=0).astype(F32)
    ls, q, op, rgb = _draw_appearance(rng, n)
    return Scene(mean, ls, q, op, rgb)


def tracking_scene(n=60_000, seed=0, outlier_fraction=0.2, offset=(0.2, 0.6)) -> tuple[Scene, int]:
    """Map for the tracking workload: (1 - outlier_fraction) n surface
    Gaussians followed by the outliers.  Surface Gaussians lie on the floor
    and walls (chosen by area, 1 cm normal jitter) and are flat, as fitted
    maps of surfaces are: in-plane log-scales N(-3, 0.5^2), 5 mm along the
    normal, a uniform random rotation about the normal.  Outliers are surface
    points pushed into the room along the inward normal by a distance uniform
    in `offset` metres (badly placed geometry a map keeps from earlier frames)
    with the isotropic appearance of _draw_appearance.  Opacity logits N(0, 1)
    and RGB uniform for all.  Returns (scene, number of surface Gaussians)."""
    rng = np.random.default_rng(seed)
    n_out = int(round(outlier_fraction * n))
    n_surf = n - n_out
    lo = np.array([_ROOM["x"][0], _ROOM["y"][0], _ROOM["z"][0]])
    hi = np.array([_ROOM["x"][1], _ROOM["y"][1], _ROOM["z"][1]])
    centre = 0.5 * (lo + hi)
    p = _AREAS / _AREAS.sum()
    # surfaces
    which = rng.choice(len(_SURFACES), size=n_surf, p=p)
    surf = lo + rng.random(size=(n_surf, 3)) * (hi - lo)
    jitter = rng.normal(0.0, 0.01, size=n_surf)
    ls_s = rng.normal(-3.0, 0.5, size=(n_surf, 3))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_surf)
    q_s = np.zeros((n_surf, 4))
    q_s[:, 0] = np.cos(0.5 * theta)
    for k, (_, axis, value) in enumerate(_SURFACES):
        sel = which == k
        surf[sel, axis] = value + jitter[sel]
        ls_s[sel, axis] = math.log(0.005)
        q_s[sel, 1 + axis] = np.sin(0.5 * theta[sel])
    # outliers
    which_o = rng.choice(len(_SURFACES), size=n_out, p=p)
    out = lo + rng.random(size=(n_out, 3)) * (hi - lo)
    dist = rng.uniform(offset[0], offset[1], size=n_out)
    for k, (_, axis, value) in enumerate(_SURFACES):
        sel = which_o == k
        out[sel, axis] = value - np.sign(value - centre[axis]) * dist[sel]
    ls_o, q_o, _, _ = _draw_appearance(rng, n_out)
    op = rng.normal(0.0, 1.0, size=n)
    rgb = rng.random(size=(n, 3))
    mean = np.concatenate([surf, out], axis=0).astype(F32)
    ls = np.concatenate([ls_s, ls_o], axis=0).astype(F32)
    q = np.concatenate([q_s, q_o], axis=0).astype(F32)
    return Scene(mean, ls, q, op.astype(F32), rgb.astype(F32)), n_surf


def subset(scene: Scene, idx) -> Scene:
    idx = np.asarray(idx)
    return Scene(*(a[idx].copy() for a in scene.arrays()), sh=None if scene.sh is None else scene.sh[idx].copy())


# --------------------------------------------------------------------------- cameras

def camera_small() -> Camera:
    """160x120, fx = fy = 150, principal point at the image centre, identity pose."""
    R, t = _identity_pose()
    return Camera(150.0, 150.0, 79.5, 59.5, R, t, 160, 120)


def camera_replica() -> Camera:
    """1200x680, f = 600 (Replica-like), identity pose: the camera sits 0.5 m
    inside the front wall of the room box looking along +z."""
    R, t = _identity_pose()
    return Camera(600.0, 600.0, 599.5, 339.5, R, t, 1200, 680)


def camera_tum() -> Camera:
    """640x480, f = 517.3, c = (318.6, 255.3) (TUM-like), identity pose."""
    R, t = _identity_pose()
    return Camera(517.3, 517.3, 318.6, 255.3, R, t, 640, 480)


def _rescaled(cam: Camera, factor: int) -> Camera:
    """Intrinsics for an image `factor` times smaller: f' = f/k and
    c' = (c + 0.5)/k - 0.5 (pixel centres at integers)."""
    return cam.with_size(cam.fx / factor, cam.fy / factor,
                         (cam.cx + 0.5) / factor - 0.5, (cam.cy + 0.5) / factor - 0.5,
                         cam.width // factor, cam.height // factor)


def camera_tum_coarse() -> Camera:
    """160x120 coarse tracking camera derived from camera_tum()."""
    return _rescaled(camera_tum(), 4)


def camera_quarter_tum() -> Camera:
    """320x240 keyframe camera derived from camera_tum()."""
    return _rescaled(camera_tum(), 2)


def camera_hyp_half() -> Camera:
    """600x340, f = 300, c = (299.5, 169.5) (half-resolution Replica-like)."""
    R, t = _identity_pose()
    return Camera(300.0, 300.0, 299.5, 169.5, R, t, 600, 340)


# --------------------------------------------------------------------------- poses

def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """SE(3) exponential of xi = (rho, phi) (translation first), float64 4x4."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    th = float(np.linalg.norm(phi))
    K = _hat(phi)
    if th < 1e-12:
        Rm = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        a = math.sin(th) / th
        b = (1.0 - math.cos(th)) / th ** 2
        c = (th - math.sin(th)) / th ** 3
        Rm = np.eye(3) + a * K + b * K @ K
        V = np.eye(3) + b * K + c * K @ K
    T = np.eye(4)
    T[:3, :3] = Rm
    T[:3, 3] = V @ rho
    return T


def perturb_pose(cam: Camera, xi) -> Camera:
    """Left-perturbed camera: T_cw <- Exp(xi) T_cw."""
    T = np.eye(4)
    T[:3, :3] = cam.R.astype(np.float64)
    T[:3, 3] = cam.t.astype(np.float64)
    T2 = se3_exp(xi) @ T
    return cam.with_pose(T2[:3, :3], T2[:3, 3])


def _look_at(centre, target, roll):
    z = target - centre
    z = z / np.linalg.norm(z)
    down = np.array([0.0, 1.0, 0.0])
    x = np.cross(down, z)
    if np.linalg.norm(x) < 1e-6:
        x = np.array([1.0, 0.0, 0.0])
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    c, s = math.cos(roll), math.sin(roll)
    x2 = c * x + s * y
    y2 = -s * x + c * y
    R = np.stack([x2, y2, z], axis=0)
    t = -R @ centre
    return R, t


def camera_tracking() -> Camera:
    """camera_tum() intrinsics at a pose that sees the floor, the back wall and
    the right wall: centre (0.5, 0.3, 0.8), looking at the floor corner
    (3, 1.5, 3.5), no roll."""
    R, t = _look_at(np.array([0.5, 0.3, 0.8]), np.array([3.0, 1.5, 3.5]), 0.0)
    return camera_tum().with_pose(R, t)


def mapping_views(seed=2):
    """Sixteen keyframes of mixed resolution inside the room box: 4 x 320x240,
    8 x 640x480 and 4 x 1200x680.  Centres are uniform in the box shrunk by
    0.5 m; each camera looks at a random surface point at least 1.5 m away with
    up close to -y and a N(0, 5 deg) roll."""
    rng = np.random.default_rng(seed)
    kinds = [camera_quarter_tum()] * 4 + [camera_tum()] * 8 + [camera_replica()] * 4
    views = []
    lo = np.array([-2.5, -1.0, 0.0])
    hi = np.array([2.5, 1.0, 3.0])
    for base in kinds:
        centre = lo + rng.random(3) * (hi - lo)
        while True:
            target = _surface_points(rng, 1, offset_sd=0.0)[0]
            if np.linalg.norm(target - centre) >= 1.5:
                break
        roll = math.radians(rng.normal(0.0, 5.0))
        R, t = _look_at(centre, target, roll)
        views.append(base.with_pose(R, t))
    return views


def hypothesis_views(seed=2, n_half=64, n_full=8, base: Camera | None = None):
    """Pose hypotheses around a base pose: Exp(delta) T_base with
    delta_rho ~ N(0, (5 cm/sqrt 3)^2 I) and delta_phi ~ N(0, (2 deg/sqrt 3)^2 I);
    `n_half` views at 600x340 followed by `n_full` at 1200x680."""
    rng = np.random.default_rng(seed)
    base = base or camera_replica()
    out = []
    for k in range(n_half + n_full):
        rho = rng.normal(0.0, 0.05 / math.sqrt(3.0), 3)
        phi = rng.normal(0.0, math.radians(2.0) / math.sqrt(3.0), 3)
        cam = perturb_pose(base, np.concatenate([rho, phi]))
        if k < n_half:
            h = camera_hyp_half()
            cam = cam.with_size(h.fx, h.fy, h.cx, h.cy, h.width, h.height)
        out.append(cam)
    return out


def tracking_start(seed=2, truth: Camera | None = None, trans=0.02, rot_deg=1.0) -> Camera:
    """Truth pose perturbed by `trans` metres along a random direction and
    `rot_deg` degrees about a random axis (left perturbation)."""
    rng = np.random.default_rng(seed)
    truth = truth or camera_tum()
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    return perturb_pose(truth, np.concatenate([trans * d, math.radians(rot_deg) * a]))


# --------------------------------------------------------------------------- images

def upstream_grads(sizes, seed=1, w_rgb=1.0, w_depth=0.1, t_scale=0.1, zero_fraction=0.05):
    """Upstream gradients shaped like an L1 loss gradient for views of the given
    (width, height) sizes, concatenated view after view: g_rgb [3*sum(HW)]
    (per view [3][H][W]) in {-w_rgb, 0, +w_rgb}, g_depth [sum(HW)] in
    {-w_depth, 0, +w_depth}, g_T [sum(HW)] ~ N(0, t_scale^2)."""
    rng = np.random.default_rng(seed)
    npx = sum(int(w) * int(h) for w, h in sizes)
    s_rgb = rng.choice(np.array([-1.0, 1.0]), size=3 * npx)
    s_rgb[rng.random(3 * npx) < zero_fraction] = 0.0
    s_d = rng.choice(np.array([-1.0, 1.0]), size=npx)
    s_d[rng.random(npx) < zero_fraction] = 0.0
    g_T = rng.normal(0.0, t_scale, size=npx)
    return (w_rgb * s_rgb).astype(F32), (w_depth * s_d).astype(F32), g_T.astype(F32)


def random_targets(sizes, seed=1, depth_range=(0.5, 4.0), invalid_fraction=0.1):
    """Target images for the L1 loss: RGB uniform in [0,1], depth uniform in
    `depth_range` with `invalid_fraction` of the pixels set to 0 (no reading),
    and a pixel mask (uint8, 1 = use the pixel)."""
    rng = np.random.default_rng(seed)
    npx = sum(int(w) * int(h) for w, h in sizes)
    rgb = rng.random(3 * npx).astype(F32)
    depth = rng.uniform(depth_range[0], depth_range[1], size=npx).astype(F32)
    depth[rng.random(npx) < invalid_fraction] = 0.0
    mask = np.ones(npx, np.uint8)
    return rgb, depth, mask


def loss_images(sizes, seed=3):
    """Per-pixel loss images (float32 [sum HW], view after view) and a pixel
    mask for the loss-median selection, one flavour per view in turn:
    exponential values (long upper tail), values rounded to quarters (ties),
    many zeros with some -0 and negative values, values with +inf and NaN
    sprinkled in.  The mask keeps ~70% of the pixels, except that views
    2, 7, 12, ... have none."""
    rng = np.random.default_rng(seed)
    vals, masks = [], []
    for v, (w, h) in enumerate(sizes):
        n = int(w) * int(h)
        kind = v % 4
        if kind == 0:
            x = rng.exponential(0.3, n)
        elif kind == 1:
            x = np.round(rng.exponential(1.0, n) * 4.0) / 4.0
        elif kind == 2:
            x = rng.exponential(0.5, n) * (rng.random(n) < 0.4)
            x[rng.random(n) < 0.05] = -0.0
            neg = rng.random(n) < 0.05
            x[neg] = -rng.uniform(0.1, 2.0, size=int(neg.sum()))
        else:
            x = rng.exponential(2.0, n)
            x[rng.random(n) < 0.02] = np.inf
            x[rng.random(n) < 0.02] = np.nan
        m = (rng.random(n) < 0.7).astype(np.uint8)
        if v % 5 == 2:
            m[:] = 0
        vals.append(x.astype(F32))
        masks.append(m)
    return np.concatenate(vals), np.concatenate(masks)


def noisy_targets(rgb, depth, seed=1, sigma=0.05, min_alpha=None, alpha=None):
    """Targets made from rendered images: C* = C + N(0, sigma^2) and
    D* = D (1 + N(0, sigma^2)); depth is set to 0 where `alpha` < `min_alpha`."""
    rng = np.random.default_rng(seed)
    t_rgb = (rgb + rng.normal(0.0, sigma, size=rgb.shape)).astype(F32)
    t_d = (depth * (1.0 + rng.normal(0.0, sigma, size=depth.shape))).astype(F32)
    if min_alpha is not None and alpha is not None:
        t_d[alpha < min_alpha] = 0.0
    return t_rgb, t_d


def expansion_images(sizes, seed=4, plant_tau_T=None, plant_tau_D=None, invalid_fraction=0.1,
                     depth_range=(0.5, 4.0)):
    """Inputs of the map-expansion adding step for views of the given sizes,
    concatenated view after view (float32): final transmittance T [sum HW]
    (uniform in [0, 1], a tenth exactly 1 = empty pixels, a tenth exactly 0),
    rendered depth [sum HW] (uniform in `depth_range`), observed depth
    [sum HW] (the rendered depth plus N(0, 0.2^2) noise, `invalid_fraction`
    zeros, a few NaN) and observed colour [3 * sum HW] (uniform in [0, 1]).
    With plant_tau_T / plant_tau_D, 2 % of the pixels each are placed exactly
    on a threshold: T = 1 - plant_tau_T, or rendered depth 1.0 and observed
    depth 1.0 + plant_tau_D (both exact in float32 for dyadic thresholds)."""
    rng = np.random.default_rng(seed)
    npx = sum(int(w) * int(h) for w, h in sizes)
    T = rng.random(npx)
    u = rng.random(npx)
    T[u < 0.1] = 1.0
    T[(u >= 0.1) & (u < 0.2)] = 0.0
    dr = rng.uniform(depth_range[0], depth_range[1], size=npx)
    do = dr + rng.normal(0.0, 0.2, size=npx)
    do[rng.random(npx) < invalid_fraction] = 0.0
    do[rng.random(npx) < 0.005] = np.nan
    rgb = rng.random(3 * npx)
    if plant_tau_T is not None:
        sel = rng.random(npx) < 0.02
        T[sel] = 1.0 - float(plant_tau_T)
    if plant_tau_D is not None:
        sel = rng.random(npx) < 0.02
        dr[sel] = 1.0
        do[sel] = 1.0 + float(plant_tau_D)
    return T.astype(F32), dr.astype(F32), do.astype(F32), rgb.astype(F32)


def room_depth(cam: Camera, seed=5, invalid_fraction=0.05):
    """Observed depth image [H*W] float32 of the empty room box (its floor,
    ceiling and walls) seen from a camera inside it: per pixel, the
    camera-frame depth at which the pixel's ray leaves the box, with
    `invalid_fraction` of the readings removed (0).  A geometric stand-in for
    a depth sensor; it evaluates nothing of the renderer."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64).reshape(3)
    o = -R.T @ t
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    d_cam = np.stack([(px - cam.cx) / cam.fx, (py - cam.cy) / cam.fy, np.ones(px.shape)], axis=-1)
    w = d_cam @ R  # world direction with unit camera-frame depth
    lo = np.array([-3.0, -1.5, -0.5])
    hi = np.array([3.0, 1.5, 3.5])
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(w > 0, (hi - o) / w, np.where(w < 0, (lo - o) / w, np.inf))
    depth = s.min(axis=-1).reshape(-1)
    rng = np.random.default_rng(seed)
    depth[rng.random(depth.size) < invalid_fraction] = 0.0
    return depth.astype(F32)


def with_sh(scene: Scene, seed=6, dc=(0.0, 2.0), sd=0.3) -> Scene:
    """A copy of `scene` with degree-1 spherical-harmonic colour coefficients
    [N, 4, 3] float32: the constant coefficient of each channel uniform in
    `dc`, the three degree-1 coefficients N(0, sd^2) (in that draw order)."""
    rng = np.random.default_rng(seed)
    sh = np.empty((scene.n, 4, 3))
    sh[:, 0, :] = rng.uniform(dc[0], dc[1], size=(scene.n, 3))
    sh[:, 1:, :] = rng.normal(0.0, sd, size=(scene.n, 3, 3))
    return dataclasses.replace(scene, sh=sh.astype(F32))
