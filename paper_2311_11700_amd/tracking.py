"""Coarse-to-fine camera tracking driver on top of the renderer (GS-SLAM
Sec. 3.3, Alg. 1): T_c coarse iterations at reduced resolution, then T_f
full-resolution iterations restricted to reliable Gaussians, each iteration
one fused forward + L1 + pose-only backward call followed by an Adam step on
the se(3) increment and a left update of the camera pose.

The fine stage renders only the reliable Gaussians of Eq. 12, selected once
with the coarse pose and the observed depth (gsr_select_reliable).  Pixels
whose loss exceeds `median_factor` times the median pixel loss are left out
(implementation details of the paper); the median is the one of the previous
iteration's pixel losses (gsr_loss_median after each fused step), since the
fused step computes the loss and the backward in one pass; the first
iteration of each stage uses no cap.  The pose is kept on the device: the
Adam step, the SE(3) exponential and the packing of the camera struct are
small torch operations, so an iteration never synchronises with the host.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import _abi as A
from .renderer import Config, Gaussians, Renderer, pack_cameras


def _hat(w: torch.Tensor) -> torch.Tensor:
    z = torch.zeros((), dtype=w.dtype, device=w.device)
    return torch.stack([torch.stack([z, -w[2], w[1]]), torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    """4x4 SE(3) exponential of xi = (rho, phi) (float64 on the device)."""
    rho, phi = xi[:3], xi[3:]
    th2 = (phi * phi).sum()
    th = torch.sqrt(th2 + 1e-30)
    K = _hat(phi)
    small = th2 < 1e-12
    a = torch.where(small, 1.0 - th2 / 6.0, torch.sin(th) / th)
    b = torch.where(small, 0.5 - th2 / 24.0, (1.0 - torch.cos(th)) / (th2 + 1e-30))
    c = torch.where(small, 1.0 / 6.0 - th2 / 120.0, (th - torch.sin(th)) / (th2 * th + 1e-30))
    I = torch.eye(3, dtype=xi.dtype, device=xi.device)
    KK = K @ K
    R = I + a * K + b * KK
    V = I + b * K + c * KK
    T = torch.eye(4, dtype=xi.dtype, device=xi.device)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


@dataclasses.dataclass
class TrackingConfig:
    coarse_iters: int = 5          # T_c (implementation details: five coarse iterations)
    fine_iters: int = 95
    lr_rho: float = 2e-4           # translation learning rate
    lr_phi: float = 5e-4           # rotation learning rate
    w_rgb: float = 0.8             # photometric weight
    w_depth: float = 0.3           # geometric weight
    coarse_factor: int = 4         # 640x480 -> 160x120
    reliable_eps: float = 0.1      # Eq. 12: keep Gaussians with |D_obs - z| <= eps (metres)
    reliable_opacity: Optional[float] = None  # optional extra rule: sigmoid(opacity) above this
    median_factor: Optional[float] = 10.0  # drop pixels above this x the median pixel loss (None: keep all)


def downsample_targets(rgb: torch.Tensor, depth: torch.Tensor, width: int, height: int, k: int):
    """k x k box averages of planar rgb [3*H*W] and depth [H*W]; depth averages
    only valid (> 0) readings."""
    h2, w2 = height // k, width // k
    c = rgb.reshape(3, height, width)[:, :h2 * k, :w2 * k].reshape(3, h2, k, w2, k).mean(dim=(2, 4))
    d = depth.reshape(height, width)[:h2 * k, :w2 * k].reshape(h2, k, w2, k)
    valid = (d > 0).to(d.dtype)
    cnt = valid.sum(dim=(1, 3))
    dd = torch.where(cnt > 0, (d * valid).sum(dim=(1, 3)) / cnt.clamp(min=1), torch.zeros_like(cnt))
    return c.reshape(-1).contiguous(), dd.reshape(-1).contiguous()


class Tracker:
    """Pose-only tracking of one frame against a fixed Gaussian map."""

    def __init__(self, gaussians: Gaussians, cam_template, cfg: Optional[TrackingConfig] = None,
                 render_cfg: Optional[Config] = None, device: int = 0):
        self.g = gaussians
        self.cfg = cfg or TrackingConfig()
        rc = render_cfg or Config()
        # Pose only; each step writes the pose gradient and loss afresh.
        self.rcfg = dataclasses.replace(rc, flags=A.GSR_POSE_GRAD | A.GSR_GRAD_OVERWRITE)
        self.cam = cam_template
        k = self.cfg.coarse_factor
        self.coarse_cam = dataclasses.replace(
            cam_template, fx=cam_template.fx / k, fy=cam_template.fy / k, cx=(cam_template.cx + 0.5) / k - 0.5,
            cy=(cam_template.cy + 0.5) / k - 0.5, width=cam_template.width // k, height=cam_template.height // k)
        self.fine = Renderer(device)
        self.fine.plan(gaussians.n, [(cam_template.width, cam_template.height)])
        self.coarse = Renderer(device)
        self.coarse.plan(gaussians.n, [(self.coarse_cam.width, self.coarse_cam.height)])
        dev = self.fine.device
        self.g_sel = gaussians
        if self.cfg.reliable_opacity is not None:
            op_mask = (torch.sigmoid(gaussians.opacity_logit) > self.cfg.reliable_opacity).to(torch.uint8)
            if gaussians.mask is not None:
                op_mask = op_mask & gaussians.mask
            self.g_sel = dataclasses.replace(gaussians, mask=op_mask.contiguous())
        self.reliable = torch.empty(gaussians.n, dtype=torch.uint8, device=dev)
        self.g_fine = dataclasses.replace(gaussians, mask=self.reliable)
        self.grads = {"d_pose": torch.zeros(1, 6, device=dev)}
        self.loss = torch.zeros(1, device=dev)
        self.px_loss = {False: torch.zeros(cam_template.width * cam_template.height, device=dev),
                        True: torch.zeros(self.coarse_cam.width * self.coarse_cam.height, device=dev)}
        self.cap = torch.full((1,), float("inf"), device=dev)

    @staticmethod
    def _pack(template, T: torch.Tensor, out: torch.Tensor):
        out[0, 4:13] = T[:3, :3].reshape(9).to(torch.float32)
        out[0, 13:16] = T[:3, 3].to(torch.float32)

    def track(self, T_init: torch.Tensor, target_rgb: torch.Tensor, target_depth: torch.Tensor,
              pixel_mask: Optional[torch.Tensor] = None, losses: Optional[list] = None,
              poses: Optional[list] = None) -> torch.Tensor:
        """Optimise the world->camera pose T (4x4 float64, device) starting at
        T_init; returns the final pose.  `losses` and `poses` (optional) collect
        the per-iteration loss tensors and the pose after each update (no host
        synchronisation here)."""
        c = self.cfg
        dev = self.fine.device
        T = T_init.to(device=dev, dtype=torch.float64).clone()
        lr = torch.tensor([c.lr_rho] * 3 + [c.lr_phi] * 3, dtype=torch.float64, device=dev)
        m = torch.zeros(6, dtype=torch.float64, device=dev)
        v = torch.zeros(6, dtype=torch.float64, device=dev)
        b1, b2, eps = 0.9, 0.999, 1e-15
        ct, cd = downsample_targets(target_rgb, target_depth, self.cam.width, self.cam.height, c.coarse_factor)
        cams_c = pack_cameras([self.coarse_cam], device=dev)
        cams_f = pack_cameras([self.cam], device=dev)
        for it in range(c.coarse_iters + c.fine_iters):
            coarse = it < c.coarse_iters
            r = self.coarse if coarse else self.fine
            cams = cams_c if coarse else cams_f
            g = self.g if coarse else self.g_fine
            self._pack(None, T, cams)
            if it == c.coarse_iters:
                # Eq. 12 with the coarse pose and the observed depth.
                self.fine.select_reliable(self.g_sel, cams_f, target_depth, self.cam.width, self.cam.height,
                                          c.reliable_eps, self.rcfg.z_near, mask_out=self.reliable)
            if it == 0 or it == c.coarse_iters:
                self.cap.fill_(float("inf"))
            pm = None if coarse else pixel_mask
            px = self.px_loss[coarse]
            r.render_l1_fused(g, cams, self.rcfg, ct if coarse else target_rgb, cd if coarse else target_depth,
                              pm, c.w_rgb, c.w_depth, out={"loss": px}, grads=self.grads, loss=self.loss,
                              loss_cap=self.cap if c.median_factor is not None else None)
            if c.median_factor is not None:
                r.loss_median(px, pm, c.median_factor, cap_out=self.cap)
            if losses is not None:
                losses.append(self.loss.clone())
            gpose = self.grads["d_pose"][0].to(torch.float64)
            m = b1 * m + (1 - b1) * gpose
            v = b2 * v + (1 - b2) * gpose * gpose
            mh = m / (1 - b1 ** (it + 1))
            vh = v / (1 - b2 ** (it + 1))
            step = -lr * mh / (torch.sqrt(vh) + eps)
            T = se3_exp(step) @ T
            if poses is not None:
                poses.append(T)
        return T
