"""Plain CPU FP64 oracle of the differentiable tile-based splatting renderer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; it exists so tests, the smoke check and the benchmark's
CPU baseline can check the GPU renderer against an independent, slow and
obviously correct implementation of what the paper computes.  It shares no
code with the GPU path (the only common module is the seeded input generator
package, which holds none of the method's arithmetic).

What is computed, and where the paper defines it (GS-SLAM, arXiv 2311.11700):
  * Scene representation: Gaussians with position, covariance, opacity and
    colour (Sec. 3.1, Eq. 1); covariance factorised as R S S^T R^T with R from
    a real-first quaternion (Eq. 2; quaternion-to-rotation formula, supplement
    Sec. A, eq. q2R).  Colour is view-independent RGB (the tracking colour
    model of Sec. 3.3 and the paper's light version) or, when the scene holds
    them, degree-1 spherical harmonics with 12 coefficients per Gaussian
    (Sec. 3.1): per channel the coefficients weight the real spherical
    harmonics of degree <= 1 of the viewing direction from the camera centre
    to the Gaussian's mean (no offset, no clamp).
  * Projection: Sigma' = J W Sigma W^T J^T (Eq. 3) with J the Jacobian of the
    perspective projection (supplement Sec. A, derivative of m_i w.r.t. the
    camera-frame point; its (0,2) entry carries z^2 in the denominator) and a
    0.3 px^2 low-pass added to the diagonal; projected centre m = K X_c / z and
    depth d = z (Sec. 3.1 below Eq. 5; Sec. 3.3 below Eq. 11).
  * Tile binning and ordering: 16x16 tiles; each Gaussian covers the tiles of
    the axis-aligned box of its 3-sigma ellipse; each tile's list is sorted by
    (float32 depth bits, index) -- the "sorting the Gaussians in depth order"
    of Sec. 3.1 made exact.
  * Compositing: front-to-back alpha blending of colour (Eq. 4) and depth
    (Eq. 5), with the cumulative opacity of Sec. 3.2 (adding step) reported
    through the final transmittance, alpha = min(0.99, sigmoid(Lambda) *
    exp(-Q/2)), entries with alpha < 1/255 skipped, and a pixel stopping before
    the entry that would take its transmittance below 1e-4.
  * Gradients: the depth blending derivatives of supplement Sec. A (eq.
    grad_depth) and their colour analogue; the chain through the projection
    (supplement Sec. A, derivatives through m_i and through Sigma'); the camera
    pose as an se(3) left perturbation (exact: the Sigma' path is kept).
  * L1 losses of Eq. 6 / Eq. 10 with colour and depth weights.

Readings of points the paper leaves open are listed with the design notes of
the repository; the ones this file depends on are repeated where used.
"""
from __future__ import annotations

import dataclasses

import numpy as np

TILE = 16
F64 = np.float64


def f32(x) -> float:
    """A configuration value as the float32 number the GPU receives."""
    return float(np.float32(x))


@dataclasses.dataclass
class Config:
    """Renderer constants (the paper is silent on them; values of the 3DGS
    rasteriser the paper extends).  `full_rect` is the smooth mode used for
    finite differences: every Gaussian covers every tile of the image."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    cutoff: float = 3.0
    z_near: float = 0.2
    lowpass: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)
    full_rect: bool = False
    # Limit g on x/z and y/z inside the Jacobian of Eq. 3: +-g W/(2 fx),
    # +-g H/(2 fy) (the paper is silent; 1.3 is the cited rasteriser's
    # value).  0 evaluates Eq. 3 as printed.
    fov_guard: float = 1.3

    def as_f32(self) -> "Config":
        return dataclasses.replace(
            self, alpha_min=f32(self.alpha_min), alpha_max=f32(self.alpha_max),
            T_min=f32(self.T_min), cutoff=f32(self.cutoff), z_near=f32(self.z_near),
            lowpass=f32(self.lowpass), bg=tuple(f32(b) for b in self.bg), fov_guard=f32(self.fov_guard))

    @staticmethod
    def smooth(bg=(0.0, 0.0, 0.0)) -> "Config":
        """No thresholds, no clamp reachable for opacities below 0.95, and every
        tile in every list: the rendered image is a smooth function of the
        parameters as long as no two depths swap order."""
        return Config(alpha_min=0.0, alpha_max=1.0, T_min=0.0, bg=bg, full_rect=True)


# Real spherical harmonics of degree <= 1 (the textbook real basis, without
# the Condon-Shortley phase) of a unit direction (x, y, z): Y_0 = 1/(2 sqrt(pi))
# and (Y_1, Y_2, Y_3) = sqrt(3/(4 pi)) (y, z, x).
SH_C0 = 0.5 / np.sqrt(np.pi)
SH_C1 = np.sqrt(3.0 / (4.0 * np.pi))


def sh_basis(d):
    """[N, 4] basis values of unit directions d [N, 3]."""
    d = np.asarray(d, F64)
    return np.stack([np.full(d.shape[0], SH_C0), SH_C1 * d[:, 1], SH_C1 * d[:, 2], SH_C1 * d[:, 0]], axis=1)


# Relative margins inside which a float32 renderer may take a threshold
# decision differently from this FP64 oracle (alpha vs alpha_min, T vs T_min,
# o*G vs alpha_max).  Pixels with such a decision are reported as ambiguous.
AMBIG_ALPHA = 3e-5
AMBIG_T = 1e-4
# Distance (in tile units) of a rectangle bound to an integer below which the
# binning decision is reported as ambiguous.
AMBIG_BIN = 1e-9


# --------------------------------------------------------------------------- Eq. 2, eq. q2R

def quat_to_rotmat(q):
    """Rotation matrix of unit quaternions q = (q_r, q_i, q_j, q_k) [N,4]
    (supplement Sec. A, eq. q2R)."""
    w, x, y, z = (q[:, k] for k in range(4))
    R = np.empty(q.shape[:1] + (3, 3), F64)
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def quat_to_rotmat_grads(q):
    """dR/dq_r, dR/dq_i, dR/dq_j, dR/dq_k of eq. q2R, each [N,3,3]."""
    w, x, y, z = (q[:, k] for k in range(4))
    n = q.shape[0]
    o = np.zeros(n)

    def m(rows):
        return 2.0 * np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)

    dw = m([[o, -z, y], [z, o, -x], [-y, x, o]])
    dx = m([[o, y, z], [y, -2 * x, -w], [z, w, -2 * x]])
    dy = m([[-2 * y, x, w], [x, o, z], [-w, z, -2 * y]])
    dz = m([[-2 * z, -w, x], [w, -2 * z, y], [x, y, o]])
    return dw, dx, dy, dz


def covariance_3d(log_scale, quat):
    """Sigma = R S S^T R^T with S = diag(exp(log_scale)) and R from the
    normalised quaternion (Eq. 2).  Returns (Sigma, R, s, qhat, |q|)."""
    qn = np.linalg.norm(quat, axis=1)
    qhat = quat / np.where(qn > 0, qn, 1.0)[:, None]
    R = quat_to_rotmat(qhat)
    s = np.exp(log_scale)
    Sigma = np.einsum("nij,nj,nkj->nik", R, s * s, R)
    return Sigma, R, s, qhat, qn


# --------------------------------------------------------------------------- Eq. 3 + binning

def _as64(a):
    return np.asarray(a, dtype=F64)


def project(scene, cam, cfg: Config):
    """Per-Gaussian projection into one camera (Eq. 3, supplement Sec. A).

    Returns a dict of FP64 arrays plus the exact integer binning data: the
    tile rectangle [tx0, tx1] x [ty0, ty1], the float32 depth bits used as the
    sort key, a `valid` mask (culled Gaussians are invalid) and `bin_ambiguous`
    for Gaussians whose rectangle bound lies within AMBIG_BIN of a tile edge.
    Culling: non-finite parameter, zero quaternion, mask = 0, z <= z_near,
    det(Sigma') <= 0, or an empty rectangle.
    """
    mean, log_scale, quat, opl, rgb = (_as64(a) for a in scene.arrays())
    n = mean.shape[0]
    W = _as64(cam.R).reshape(3, 3)
    t = _as64(cam.t).reshape(3)
    fx, fy, cx, cy = (float(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    TX = (int(cam.width) + TILE - 1) // TILE
    TY = (int(cam.height) + TILE - 1) // TILE

    sh = getattr(scene, "sh", None)
    sh = None if sh is None else _as64(sh).reshape(n, 4, 3)
    finite = np.ones(n, bool)
    for a in (mean, log_scale, quat, opl[:, None], rgb if sh is None else sh.reshape(n, 12)):
        finite &= np.isfinite(a).all(axis=1)
    with np.errstate(all="ignore"):
        Sigma, Rq, s, qhat, qn = covariance_3d(log_scale, quat)
        mx, my, mz = mean[:, 0], mean[:, 1], mean[:, 2]
        # X_c = W X + t, each row summed left to right.
        x = ((W[0, 0] * mx + W[0, 1] * my) + W[0, 2] * mz) + t[0]
        y = ((W[1, 0] * mx + W[1, 1] * my) + W[1, 2] * mz) + t[1]
        z = ((W[2, 0] * mx + W[2, 1] * my) + W[2, 2] * mz) + t[2]
        zf = z.astype(np.float32)
        Sigma_c = np.einsum("ij,njk,lk->nil", W, Sigma, W)
        # Eq. 3's Jacobian with x/z, y/z limited by the guard (the projected
        # centre u, v below uses the true ratios).
        rxz, ryz = x / z, y / z
        free_x = np.ones(n, bool)
        free_y = np.ones(n, bool)
        if cfg.fov_guard > 0:
            lx = float(cfg.fov_guard) * (0.5 * float(cam.width)) / fx
            ly = float(cfg.fov_guard) * (0.5 * float(cam.height)) / fy
            free_x = ~((rxz > lx) | (rxz < -lx))
            free_y = ~((ryz > ly) | (ryz < -ly))
            rxz = np.minimum(lx, np.maximum(-lx, rxz))
            ryz = np.minimum(ly, np.maximum(-ly, ryz))
        J = np.zeros((n, 2, 3))
        J[:, 0, 0] = fx / z
        J[:, 0, 2] = -(fx * rxz) / z
        J[:, 1, 1] = fy / z
        J[:, 1, 2] = -(fy * ryz) / z
        cov2 = np.einsum("nij,njk,nlk->nil", J, Sigma_c, J)
        cov2[:, 0, 0] += cfg.lowpass
        cov2[:, 1, 1] += cfg.lowpass
        det = cov2[:, 0, 0] * cov2[:, 1, 1] - cov2[:, 0, 1] * cov2[:, 0, 1]
        conic = np.stack([cov2[:, 1, 1] / det, -cov2[:, 0, 1] / det, cov2[:, 0, 0] / det], axis=1)
        u = (fx * x) / z + cx
        v = (fy * y) / z + cy
        rx = cfg.cutoff * np.sqrt(cov2[:, 0, 0])
        ry = cfg.cutoff * np.sqrt(cov2[:, 1, 1])
        opacity = 1.0 / (1.0 + np.exp(-opl))
        sh_extra = {}
        if sh is not None:
            # Viewing direction from the camera centre o = -W^T t to the mean.
            vdir = mean + (W.T @ t)[None, :]
            vlen = np.linalg.norm(vdir, axis=1)
            dirs = vdir / vlen[:, None]
            Y = sh_basis(dirs)
            rgb = np.einsum("nk,nkc->nc", Y, sh)
            sh_extra = dict(sh=sh, sh_Y=Y, sh_dir=dirs, sh_len=vlen, t=t)

    valid = finite & (qn > 0) & (z > cfg.z_near) & (det > 0)
    if getattr(scene, "mask", None) is not None:
        valid &= np.asarray(scene.mask) != 0

    with np.errstate(all="ignore"):
        bx0, bx1 = (u - rx) / TILE, (u + rx) / TILE
        by0, by1 = (v - ry) / TILE, (v + ry) / TILE
    rect = np.zeros((n, 4), np.int64)
    amb = np.zeros(n, bool)
    if cfg.full_rect:
        rect[:] = (0, TX - 1, 0, TY - 1)
    else:
        ok = valid.copy()
        rect[ok, 0] = np.maximum(0, np.floor(bx0[ok])).astype(np.int64)
        rect[ok, 1] = np.minimum(TX - 1, np.floor(bx1[ok])).astype(np.int64)
        rect[ok, 2] = np.maximum(0, np.floor(by0[ok])).astype(np.int64)
        rect[ok, 3] = np.minimum(TY - 1, np.floor(by1[ok])).astype(np.int64)
        for b in (bx0, bx1, by0, by1):
            with np.errstate(all="ignore"):
                d = np.abs(b - np.round(b))
            amb |= ok & (d < AMBIG_BIN * np.maximum(1.0, np.abs(b)))
    valid &= (rect[:, 0] <= rect[:, 1]) & (rect[:, 2] <= rect[:, 3])
    rect[~valid] = (0, -1, 0, -1)
    return dict(
        n=n, TX=TX, TY=TY, valid=valid, rect=rect, bin_ambiguous=amb & valid,
        Xc=np.stack([x, y, z], axis=1), z=z, zbits=zf.view(np.uint32), mean_w=mean,
        Sigma=Sigma, Sigma_c=Sigma_c, Rq=Rq, s=s, qhat=qhat, qn=qn, J=J, cov2=cov2,
        conic=conic, uv=np.stack([u, v], axis=1), opacity=opacity, rgb=rgb,
        W=W, fx=fx, fy=fy, rxz=rxz, ryz=ryz, free_x=free_x, free_y=free_y, **sh_extra,
    )


def tile_lists(proj):
    """Per-tile Gaussian lists in blending order.

    Every valid Gaussian is listed in every tile of its 3-sigma rectangle
    (Sec. 3.1: the Gaussians covering a tile, sorted by depth).  Tile id =
    ty * TX + tx.  Returns (starts [TX*TY + 1], gauss [P]) where the list of
    tile k is gauss[starts[k]:starts[k+1]], ordered by (float32 depth bits,
    Gaussian index)."""
    TX, TY = proj["TX"], proj["TY"]
    rect = proj["rect"]
    idx = np.nonzero(proj["valid"])[0]
    tx0, tx1, ty0, ty1 = (rect[idx, k] for k in range(4))
    w = tx1 - tx0 + 1
    cnt = w * (ty1 - ty0 + 1)
    # One pair per tile of each rectangle, row-major inside the rectangle.
    gauss = np.repeat(idx, cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    j = np.arange(gauss.size) - first
    ww = np.repeat(w, cnt)
    tiles_g = (np.repeat(ty0, cnt) + j // ww) * TX + np.repeat(tx0, cnt) + j % ww
    order = np.lexsort((gauss, proj["zbits"][gauss], tiles_g))
    tiles_g, gauss = tiles_g[order], gauss[order]
    starts = np.searchsorted(tiles_g, np.arange(TX * TY + 1), side="left")
    return starts, gauss


def tile_alpha_max(proj, tile, lst, width, height, cfg: Config):
    """For each Gaussian of `lst`, the largest alpha = min(alpha_max,
    o exp(-Q/2)) it reaches at a pixel centre of tile `tile` inside the
    image (FP64, every pixel evaluated).  A Gaussian whose value is below
    alpha_min is skipped by every pixel of the tile (Eq. 4-5 blend only
    entries with alpha >= alpha_min), so a renderer may leave it out of the
    tile's list without changing any output."""
    lst = np.asarray(lst, np.int64)
    if lst.size == 0:
        return np.zeros(0)
    px, py = _tile_pixels(tile, proj["TX"], width, height)
    u, v = proj["uv"][lst, 0], proj["uv"][lst, 1]
    a, b, c = (proj["conic"][lst, k] for k in range(3))
    dx = u[None, :] - px[:, None].astype(F64)
    dy = v[None, :] - py[:, None].astype(F64)
    Q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    alpha = np.minimum(cfg.alpha_max, proj["opacity"][lst][None, :] * np.exp(-0.5 * Q))
    return alpha.max(axis=0)


# --------------------------------------------------------------------------- Eq. 4-5

def _tile_pixels(tile, TX, width, height):
    ty, tx = divmod(int(tile), TX)
    py, px = np.meshgrid(np.arange(ty * TILE, ty * TILE + TILE), np.arange(tx * TILE, tx * TILE + TILE),
                         indexing="ij")
    px, py = px.ravel(), py.ravel()
    inside = (px < width) & (py < height)
    return px[inside], py[inside]


def _blend_tile(proj, lst, px, py, cfg: Config):
    """Front-to-back blending (Eq. 4-5) of the Gaussians `lst` (in blending
    order) at pixels (px, py), written as products and sums over the list."""
    n, L = px.size, lst.size
    if L == 0:
        e = np.zeros((n, 0))
        return dict(C=np.tile(np.asarray(cfg.bg, F64), (n, 1)), D=np.zeros(n), Tf=np.ones(n),
                    last=np.zeros(n, np.int64), amb=np.zeros(n, bool), amb_grad=np.zeros(n, bool),
                    dx=e, dy=e, G=e, oG=e, alpha=e, clamped=e.astype(bool), contrib=e.astype(bool),
                    ac=e, Tb=e, w=e)
    u, v = proj["uv"][lst, 0], proj["uv"][lst, 1]
    a, b, c = (proj["conic"][lst, k] for k in range(3))
    o = proj["opacity"][lst]
    dx = u[None, :] - px[:, None].astype(F64)
    dy = v[None, :] - py[:, None].astype(F64)
    Q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    G = np.exp(-0.5 * Q)
    oG = o * G
    alpha = np.minimum(cfg.alpha_max, oG)
    gate = alpha >= cfg.alpha_min
    a1 = np.where(gate, alpha, 0.0)
    P = np.cumprod(1.0 - a1, axis=1)
    stop = gate & (P < cfg.T_min)
    s = np.where(stop.any(axis=1), np.argmax(stop, axis=1), L)
    pos = np.arange(L)[None, :]
    contrib = gate & (pos < s[:, None])
    ac = np.where(contrib, alpha, 0.0)
    Pc = np.cumprod(1.0 - ac, axis=1)
    Tb = np.concatenate([np.ones((n, 1)), Pc[:, :-1]], axis=1)
    Tf = Pc[:, -1]
    w = ac * Tb
    bg = np.asarray(cfg.bg, F64)
    C = w @ proj["rgb"][lst] + Tf[:, None] * bg[None, :]
    D = w @ proj["z"][lst]
    anyc = contrib.any(axis=1)
    last = np.where(anyc, L - np.argmax(contrib[:, ::-1], axis=1), 0)

    considered = pos <= s[:, None]
    amb = (considered & (np.abs(alpha - cfg.alpha_min) <= AMBIG_ALPHA * cfg.alpha_min)).any(axis=1)
    if cfg.T_min > 0:
        amb |= (considered & gate & (np.abs(P - cfg.T_min) <= AMBIG_T * cfg.T_min)).any(axis=1)
    clamped = oG > cfg.alpha_max
    amb_grad = amb | (contrib & (np.abs(oG - cfg.alpha_max) <= AMBIG_ALPHA * cfg.alpha_max)).any(axis=1)
    return dict(C=C, D=D, Tf=Tf, last=last, amb=amb, amb_grad=amb_grad,
                dx=dx, dy=dy, G=G, oG=oG, alpha=alpha, clamped=clamped, contrib=contrib,
                ac=ac, Tb=Tb, w=w)


def render(scene, cam, cfg: Config = None, tiles=None, proj=None, lists=None):
    """Render one view.  Returns dict with rgb [3,H,W], depth [H,W],
    T_final [H,W], alpha = 1 - T_final (the paper's cumulative opacity),
    last [H,W] (1 + position of the last contributing entry in the tile list,
    0 if none), ambiguous / ambiguous_grad [H,W] (threshold decisions within
    the float32 margins), and `done` [H,W] marking the pixels computed (all,
    unless `tiles` restricts the work to some tile ids)."""
    cfg = (cfg or Config()).as_f32()
    proj = proj if proj is not None else project(scene, cam, cfg)
    starts, gauss = lists if lists is not None else tile_lists(proj)
    H, Wd = int(cam.height), int(cam.width)
    TX = proj["TX"]
    out = dict(rgb=np.zeros((3, H, Wd)), depth=np.zeros((H, Wd)), T_final=np.ones((H, Wd)),
               last=np.zeros((H, Wd), np.int64), ambiguous=np.zeros((H, Wd), bool),
               ambiguous_grad=np.zeros((H, Wd), bool), done=np.zeros((H, Wd), bool))
    tiles = range(TX * proj["TY"]) if tiles is None else tiles
    for tile in tiles:
        px, py = _tile_pixels(tile, TX, Wd, H)
        lst = gauss[starts[tile]:starts[tile + 1]]
        r = _blend_tile(proj, lst, px, py, cfg)
        out["rgb"][:, py, px] = r["C"].T
        out["depth"][py, px] = r["D"]
        out["T_final"][py, px] = r["Tf"]
        out["last"][py, px] = r["last"]
        out["ambiguous"][py, px] = r["amb"]
        out["ambiguous_grad"][py, px] = r["amb_grad"]
        out["done"][py, px] = True
    out["alpha"] = 1.0 - out["T_final"]
    out["proj"], out["lists"] = proj, (starts, gauss)
    return out


# --------------------------------------------------------------------------- backward

def _blend_tile_backward(proj, lst, px, py, cfg: Config, r, gC, gD, gT):
    """Gradients of <gC, C> + <gD, D> + <gT, T_final> w.r.t. the per-entry 2D
    quantities, holding the contributor set fixed.  The derivative of the
    blend w.r.t. alpha_j is c_j T_j - (sum_{m>j} c_m alpha_m T_m + T_f bg) /
    (1 - alpha_j) (supplement eq. grad_depth for depth; the same form for
    colour), evaluated with FP64 prefix products and suffix sums."""
    rgb = proj["rgb"][lst]                 # [L,3]
    z = proj["z"][lst]                      # [L]
    a, b, c = (proj["conic"][lst, k] for k in range(3))
    w, ac, Tb, Tf = r["w"], r["ac"], r["Tb"], r["Tf"]
    contrib = r["contrib"]
    bg = np.asarray(cfg.bg, F64)

    def suffix_excl(x):  # sum over m > j along axis 1
        return np.flip(np.cumsum(np.flip(x, axis=1), axis=1), axis=1) - x

    SC = suffix_excl(w[:, :, None] * rgb[None, :, :]) + (Tf[:, None, None] * bg[None, None, :])
    SD = suffix_excl(w * z[None, :])
    inv = np.where(contrib, 1.0 / (1.0 - np.where(contrib, ac, 0.0)), 0.0)
    dC_da = rgb[None, :, :] * Tb[:, :, None] - SC * inv[:, :, None]
    dD_da = z[None, :] * Tb - SD * inv
    dT_da = -Tf[:, None] * inv
    dL_da = np.einsum("pc,pjc->pj", gC, dC_da) + gD[:, None] * dD_da + gT[:, None] * dT_da
    dL_da = np.where(contrib, dL_da, 0.0)

    dL_doG = np.where(contrib & ~r["clamped"], dL_da, 0.0)
    g_o = np.sum(dL_doG * r["G"], axis=0)
    dL_dQ = dL_doG * (-0.5 * r["oG"])
    dx, dy = r["dx"], r["dy"]
    g_u = np.sum(dL_dQ * 2.0 * (a * dx + b * dy), axis=0)
    g_v = np.sum(dL_dQ * 2.0 * (b * dx + c * dy), axis=0)
    g_a = np.sum(dL_dQ * dx * dx, axis=0)
    g_b = np.sum(dL_dQ * 2.0 * dx * dy, axis=0)
    g_c = np.sum(dL_dQ * dy * dy, axis=0)
    g_rgb = np.einsum("pc,pj->jc", gC, w)
    g_z = np.sum(gD[:, None] * w, axis=0)
    return np.stack([g_u, g_v, g_a, g_b, g_c, g_o, g_rgb[:, 0], g_rgb[:, 1], g_rgb[:, 2], g_z], axis=1)


GRAD2D_FIELDS = ("u", "v", "conic_a", "conic_b", "conic_c", "opacity", "r", "g", "b", "depth")


def backward_2d(scene, cam, cfg: Config, g_rgb, g_depth, g_T, fwd=None, tiles=None):
    """Per-Gaussian gradients w.r.t. (u, v, conic a, b, c, opacity, r, g, b,
    depth), summed over every pixel of the view (or of the tiles listed in
    `tiles`: exact for Gaussians whose rectangle lies inside them).  Upstream
    gradients are images g_rgb [3,H,W], g_depth [H,W], g_T [H,W] (g_T may be
    None)."""
    cfg = (cfg or Config()).as_f32()
    fwd = fwd if fwd is not None else render(scene, cam, cfg)
    proj = fwd["proj"]
    starts, gauss = fwd["lists"]
    H, Wd = int(cam.height), int(cam.width)
    g_rgb = np.asarray(g_rgb, F64).reshape(3, H, Wd)
    g_depth = np.asarray(g_depth, F64).reshape(H, Wd)
    g_T = np.zeros((H, Wd)) if g_T is None else np.asarray(g_T, F64).reshape(H, Wd)
    g2 = np.zeros((proj["n"], 10))
    for tile in (range(proj["TX"] * proj["TY"]) if tiles is None else tiles):
        lst = gauss[starts[tile]:starts[tile + 1]]
        if lst.size == 0:
            continue
        px, py = _tile_pixels(tile, proj["TX"], Wd, H)
        r = _blend_tile(proj, lst, px, py, cfg)
        gl = _blend_tile_backward(proj, lst, px, py, cfg, r, g_rgb[:, py, px].T, g_depth[py, px], g_T[py, px])
        np.add.at(g2, lst, gl)
    return g2, fwd


def sigma2d_backward(G2, J, Sc):
    """Gradients of Sigma' = J Sigma_c J^T: given dL/dSigma' (symmetric [N,2,2])
    return (dL/dSigma_c = J^T G J, dL/dJ = 2 G J Sigma_c) (Eq. 3)."""
    GSc = np.einsum("nji,njk,nkl->nil", J, G2, J)
    GJ = 2.0 * np.einsum("nij,njk,nkl->nil", G2, J, Sc)
    return GSc, GJ


def backward_params(proj, g2, cfg: Config, approx_pose=False, pose_q=None):
    """Chain the 2D gradients to the Gaussian parameters and the camera pose
    (supplement Sec. A).  Pose gradient: left perturbation T_cw <- Exp(xi) T_cw
    with xi = (rho, phi), evaluated at xi = 0.  `approx_pose` drops the Sigma'
    path from the pose gradient only, as the paper does for speed.
    With pose_q (the camera's quaternion, R = R(q / |q|)), also the gradient
    in the paper's pose parameters: pose_t = sum_i dL/dX_c,i (X_c = R X + t)
    and pose_q through dX_c/dq = (dR/dq) X (eq. grad_q) and, unless
    approx_pose, the camera-frame covariance R Sigma R^T; projected onto the
    tangent of the normalisation.
    Returns dict(mean, log_scale, quat, opacity_logit, rgb, pose[6]
    [, pose_q[4], pose_t[3]])."""
    n = proj["n"]
    v = proj["valid"]
    g_u, g_v, g_a, g_b, g_c, g_o = (g2[:, k] for k in range(6))
    g_rgb, g_zd = g2[:, 6:9], g2[:, 9]
    fx, fy = proj["fx"], proj["fy"]
    x, y, z = (proj["Xc"][:, k] for k in range(3))
    W = proj["W"]
    a, b, c = (proj["conic"][:, k] for k in range(3))
    J, Sc = proj["J"], proj["Sigma_c"]

    M = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    GM = np.stack([np.stack([g_a, 0.5 * g_b], -1), np.stack([0.5 * g_b, g_c], -1)], -2)
    G2 = -np.einsum("nij,njk,nkl->nil", M, GM, M)          # dL/dSigma'
    GSc, GJ = sigma2d_backward(G2, J, Sc)

    # J02 = -fx r/z with r = x/z while x/z is inside the guard (then
    # dJ02/dx = -fx/z^2, dJ02/dz = 2 fx x/z^3) and r = its limit outside it
    # (dJ02/dx = 0, dJ02/dz = fx r/z^2); J12 likewise.
    fxm, fym = proj["free_x"].astype(np.float64), proj["free_y"].astype(np.float64)
    rxz, ryz = proj["rxz"], proj["ryz"]
    gX = np.zeros((n, 3))
    gX[:, 0] = g_u * fx / z + GJ[:, 0, 2] * (-fx / (z * z)) * fxm
    gX[:, 1] = g_v * fy / z + GJ[:, 1, 2] * (-fy / (z * z)) * fym
    dJ02_dz = np.where(fxm > 0, 2.0 * fx * x / z ** 3, fx * rxz / (z * z))
    dJ12_dz = np.where(fym > 0, 2.0 * fy * y / z ** 3, fy * ryz / (z * z))
    gX[:, 2] = (g_u * (-fx * x / (z * z)) + g_v * (-fy * y / (z * z))
                + GJ[:, 0, 0] * (-fx / (z * z)) + GJ[:, 0, 2] * dJ02_dz
                + GJ[:, 1, 1] * (-fy / (z * z)) + GJ[:, 1, 2] * dJ12_dz + g_zd)

    g_mean = gX @ W                                          # W^T gX per row
    GS = np.einsum("ji,njk,kl->nil", W, GSc, W)              # W^T GSc W
    Rq, s = proj["Rq"], proj["s"]
    s2 = s * s
    GR = 2.0 * np.einsum("nij,njk,nk->nik", GS, Rq, s2)      # 2 G_Sigma R S^2
    RtGR = np.einsum("nji,njk,nkl->nil", Rq, GS, Rq)
    g_s = 2.0 * s * np.einsum("nii->ni", RtGR)
    g_ls = s * g_s
    dR = quat_to_rotmat_grads(proj["qhat"])
    g_qhat = np.stack([np.einsum("nij,nij->n", GR, d) for d in dR], axis=1)
    qhat, qn = proj["qhat"], proj["qn"]
    g_q = (g_qhat - qhat * np.sum(qhat * g_qhat, axis=1, keepdims=True)) / np.where(qn > 0, qn, 1.0)[:, None]
    o = proj["opacity"]
    g_op = g_o * o * (1.0 - o)

    if approx_pose:
        gXp = np.zeros((n, 3))
        gXp[:, 0] = g_u * fx / z
        gXp[:, 1] = g_v * fy / z
        gXp[:, 2] = g_u * (-fx * x / (z * z)) + g_v * (-fy * y / (z * z)) + g_zd
        A = np.zeros((n, 3, 3))
    else:
        gXp = gX
        A = np.einsum("nij,njk->nik", Sc, GSc) - np.einsum("nij,njk->nik", GSc, Sc)
    # Degree-1 spherical-harmonic colour: dL/dcoefficients = Y (x) dL/dc, and
    # through the viewing direction d = vdir / |vdir|, vdir = mean - o:
    # dL/dvdir = (I - d d^T) dL/dd / |vdir|, which moves with the mean and
    # against the camera centre (a left perturbation moves o by -W^T rho).
    g_sh = None
    g_vdir = np.zeros((n, 3))
    if "sh" in proj:
        Y, d, sh = proj["sh_Y"], proj["sh_dir"], proj["sh"]
        g_sh = Y[:, :, None] * g_rgb[:, None, :]
        gY = np.einsum("nkc,nc->nk", sh, g_rgb)
        g_d = SH_C1 * np.stack([gY[:, 3], gY[:, 1], gY[:, 2]], axis=1)
        g_vdir = (g_d - d * np.sum(d * g_d, axis=1, keepdims=True)) / proj["sh_len"][:, None]
        g_mean = g_mean + g_vdir
    Xc = proj["Xc"]
    rho = np.sum(gXp[v], axis=0) + W @ np.sum(g_vdir[v], axis=0)
    phi_pts = np.cross(Xc[v], gXp[v])
    phi_cov = np.stack([A[v, 1, 2] - A[v, 2, 1], A[v, 2, 0] - A[v, 0, 2], A[v, 0, 1] - A[v, 1, 0]], axis=1)
    phi = np.sum(phi_pts + phi_cov, axis=0)

    def z0(arr):
        arr = np.where(v.reshape((-1,) + (1,) * (arr.ndim - 1)), arr, 0.0)
        return arr

    out = dict(mean=z0(g_mean), log_scale=z0(g_ls), quat=z0(g_q), opacity_logit=z0(g_op),
               rgb=z0(g_rgb), pose=np.concatenate([rho, phi]))
    if g_sh is not None:
        out["sh"] = z0(g_sh)
    if pose_q is not None:
        cq = np.asarray(pose_q, np.float64).reshape(1, 4)
        cqn = float(np.linalg.norm(cq))
        cqh = cq / cqn
        Rc = quat_to_rotmat(cqh)[0]
        dRc = [d[0] for d in quat_to_rotmat_grads(cqh)]
        g_qh = np.zeros(4)
        for k in range(4):
            # centre: dX_c/dq_k = (dR/dq_k) X for the world point X
            Xw = proj["mean_w"][v]
            g_qh[k] = np.sum(gXp[v] * (Xw @ dRc[k].T))
            if not approx_pose:
                # covariance: d(R Sigma R^T) = dR Sigma R^T + R Sigma dR^T
                S = proj["Sigma"][v]
                dSc = np.einsum("ij,njk,lk->nil", dRc[k], S, Rc) + np.einsum("ij,njk,lk->nil", Rc, S, dRc[k])
                g_qh[k] += np.sum(GSc[v] * dSc)
            if "sh" in proj:
                # viewing directions: vdir = mean + R^T t moves by (dR/dq_k)^T t
                g_qh[k] += float(np.sum(g_vdir[v] @ (dRc[k].T @ proj["t"])))
        out["pose_q"] = (g_qh - cqh[0] * float(cqh[0] @ g_qh)) / cqn
        out["pose_t"] = np.sum(gXp[v], axis=0) + Rc @ np.sum(g_vdir[v], axis=0)
    return out


def render_backward(scene, cam, cfg: Config, g_rgb, g_depth, g_T=None, approx_pose=False, fwd=None):
    """Gradients of <g_rgb, C> + <g_depth, D> + <g_T, T_final> for one view."""
    cfg = (cfg or Config()).as_f32()
    g2, fwd = backward_2d(scene, cam, cfg, g_rgb, g_depth, g_T, fwd=fwd)
    out = backward_params(fwd["proj"], g2, cfg, approx_pose=approx_pose)
    out["grad2d"] = g2
    out["fwd"] = fwd
    return out


# --------------------------------------------------------------------------- Eq. 6 / 10

def l1_pixel_loss(rgb, depth, target_rgb, target_depth, pixel_mask=None, w_rgb=1.0, w_depth=0.1):
    """Each pixel's own term of the L1 loss: w_rgb sum_c |C_c - C*_c| +
    w_depth [D* > 0] |D - D*|, 0 where pixel_mask is 0.  [H, W] FP64."""
    rgb = np.asarray(rgb, F64)
    depth = np.asarray(depth, F64)
    trgb = np.asarray(target_rgb, F64).reshape(rgb.shape)
    tdep = np.asarray(target_depth, F64).reshape(depth.shape)
    m = np.ones(depth.shape, bool) if pixel_mask is None else (np.asarray(pixel_mask).reshape(depth.shape) != 0)
    lp = w_rgb * np.abs(rgb - trgb).sum(axis=0) + w_depth * (tdep > 0) * np.abs(depth - tdep)
    return np.where(m, lp, 0.0)


def l1_loss(rgb, depth, target_rgb, target_depth, pixel_mask=None, w_rgb=1.0, w_depth=0.1, loss_cap=None):
    """L = w_rgb * sum |C - C*| + w_depth * sum_{D* > 0} |D - D*| over pixels
    with pixel_mask != 0 (Eq. 6 sums; Eq. 10 colour term).  With `loss_cap`,
    pixels whose own loss term exceeds it are ignored as well (the tracking
    rule of the implementation details: loss above ten times the median).
    Returns (loss, dL/dC, dL/dD) with sign(0) = 0."""
    rgb = np.asarray(rgb, F64)
    depth = np.asarray(depth, F64)
    trgb = np.asarray(target_rgb, F64).reshape(rgb.shape)
    tdep = np.asarray(target_depth, F64).reshape(depth.shape)
    m = np.ones(depth.shape) if pixel_mask is None else (np.asarray(pixel_mask).reshape(depth.shape) != 0)
    if loss_cap is not None:
        lp = l1_pixel_loss(rgb, depth, trgb, tdep, None, w_rgb, w_depth)
        m = m * (lp <= loss_cap)
    md = m * (tdep > 0)
    dc = rgb - trgb
    dd = depth - tdep
    loss = w_rgb * np.sum(m[None] * np.abs(dc)) + w_depth * np.sum(md * np.abs(dd))
    return loss, w_rgb * m[None] * np.sign(dc), w_depth * md * np.sign(dd)


def loss_median(px_loss, pixel_mask=None):
    """Lower median (the element of rank floor((m - 1) / 2) in ascending
    order) of the float32 values px_loss over the m pixels with
    pixel_mask != 0; None if m = 0.  Values compare as non-negative floats:
    negative values and -0 count as 0 and NaN ranks above +inf.  One plain
    sort."""
    v = np.asarray(px_loss, np.float32).reshape(-1)
    if pixel_mask is not None:
        v = v[np.asarray(pixel_mask).reshape(-1) != 0]
    if v.size == 0:
        return None

    def key(x):
        if np.isnan(x):
            return (1, 0.0)
        return (0, max(float(x), 0.0))

    ordered = sorted(v.tolist(), key=key)
    x = ordered[(len(ordered) - 1) // 2]
    return np.float32(0.0) if (not np.isnan(x) and x <= 0.0) else np.float32(x)


def loss_cap(px_loss, pixel_mask=None, factor=10.0):
    """factor x lower median in float32 arithmetic, +inf without pixels."""
    med = loss_median(px_loss, pixel_mask)
    return np.float32(np.inf) if med is None else np.float32(np.float32(factor) * med)


# --------------------------------------------------------------------------- Eq. 12

def select_reliable(scene, cam, depth_obs, eps, z_near=0.2, mask=None):
    """Reliable-Gaussian selection of the fine tracking stage (Eq. 12): a
    Gaussian whose centre projects (in front of the camera) onto a pixel of
    the image with a valid observed depth D is kept only if |D - z| <= eps,
    z being its camera-frame depth; all other Gaussians are kept (no
    evidence), and Gaussians excluded by `mask` stay excluded.  The pixel is
    the nearest one to the projected centre.  Returns a uint8 mask."""
    mean = _as64(scene.mean)
    W = _as64(cam.R).reshape(3, 3)
    t = _as64(cam.t).reshape(3)
    depth_obs = np.asarray(depth_obs, np.float32).reshape(int(cam.height), int(cam.width))
    eps, z_near = f32(eps), f32(z_near)
    n = mean.shape[0]
    keep = np.ones(n, np.uint8) if mask is None else (np.asarray(mask) != 0).astype(np.uint8)
    for i in range(n):  # plain loop: one Gaussian at a time
        if not keep[i]:
            continue
        mx, my, mz = mean[i]
        x = ((W[0, 0] * mx + W[0, 1] * my) + W[0, 2] * mz) + t[0]
        y = ((W[1, 0] * mx + W[1, 1] * my) + W[1, 2] * mz) + t[1]
        z = ((W[2, 0] * mx + W[2, 1] * my) + W[2, 2] * mz) + t[2]
        if not z > z_near:
            continue
        u = (float(cam.fx) * x) / z + float(cam.cx)
        v = (float(cam.fy) * y) / z + float(cam.cy)
        px, py = np.floor(u + 0.5), np.floor(v + 0.5)
        if 0 <= px < int(cam.width) and 0 <= py < int(cam.height):
            D = float(depth_obs[int(py), int(px)])
            if D > 0 and abs(D - z) > eps:
                keep[i] = 0
    return keep
