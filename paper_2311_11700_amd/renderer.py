"""Thin Python binding of the C ABI (include/gsr.h) over torch device memory.

Every step of the rendering path runs in libgsr.so; this module only builds
the C structs from torch tensors, passes torch's current HIP stream, and maps
status codes to exceptions.  Method names follow the C entry points without
the ``gsr_`` prefix (``Renderer.render_forward`` calls ``gsr_render_forward``).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _abi as A


class GsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


@dataclasses.dataclass
class Config:
    """Mirror of gsr_config (renderer constants and flags)."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    cutoff_sigma: float = 3.0
    z_near: float = 0.2
    lowpass: float = 0.3
    bg: Sequence[float] = (0.0, 0.0, 0.0)
    flags: int = A.GSR_GAUSS_GRAD | A.GSR_POSE_GRAD
    fov_guard: float = 1.3

    def to_c(self) -> A.gsr_config:
        c = A.gsr_config()
        c.alpha_min, c.alpha_max, c.T_min = self.alpha_min, self.alpha_max, self.T_min
        c.cutoff_sigma, c.z_near, c.lowpass = self.cutoff_sigma, self.z_near, self.lowpass
        for k in range(3):
            c.bg[k] = float(self.bg[k])
        c.flags = int(self.flags)
        c.fov_guard = float(self.fov_guard)
        return c

    @staticmethod
    def smooth(bg=(0.0, 0.0, 0.0), flags=A.GSR_GAUSS_GRAD | A.GSR_POSE_GRAD) -> "Config":
        """Finite-difference mode: no thresholds, every tile in every list."""
        return Config(alpha_min=0.0, alpha_max=1.0, T_min=0.0, bg=bg, flags=flags | A.GSR_FULL_RECT)


@dataclasses.dataclass
class Gaussians:
    """Gaussian parameters on the device (float32, contiguous)."""
    mean: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    opacity_logit: torch.Tensor
    rgb: Optional[torch.Tensor]
    mask: Optional[torch.Tensor] = None
    # degree-1 spherical-harmonic colour [n, 4, 3]; when set, rgb is not read
    sh: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    @staticmethod
    def from_arrays(mean, log_scale, quat, opacity_logit, rgb, mask=None, device="cuda", sh=None) -> "Gaussians":
        def t(a, dt=torch.float32):
            return torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        return Gaussians(t(mean).reshape(-1, 3), t(log_scale).reshape(-1, 3), t(quat).reshape(-1, 4),
                         t(opacity_logit).reshape(-1), None if rgb is None else t(rgb).reshape(-1, 3),
                         None if mask is None else t(mask, torch.uint8).reshape(-1),
                         None if sh is None else t(sh).reshape(-1, 4, 3))

    def c(self) -> A.gsr_gaussians:
        names = ("mean", "log_scale", "quat", "opacity_logit") + (("sh",) if self.sh is not None else ("rgb",))
        for name in names:
            x = getattr(self, name)
            if x is None or x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError(f"Gaussians.{name} must be a contiguous float32 device tensor")
            per = dict(mean=3, log_scale=3, quat=4, opacity_logit=1, rgb=3, sh=12)[name]
            if x.numel() != per * self.n:
                raise ValueError(f"Gaussians.{name} holds {x.numel()} values, {per * self.n} expected")
        g = A.gsr_gaussians()
        g.n = self.n
        g.mean, g.log_scale, g.quat = self.mean.data_ptr(), self.log_scale.data_ptr(), self.quat.data_ptr()
        g.opacity_logit = self.opacity_logit.data_ptr()
        g.rgb = self.rgb.data_ptr() if self.rgb is not None else None
        g.mask = self.mask.data_ptr() if self.mask is not None else None
        g.sh = self.sh.data_ptr() if self.sh is not None else None
        return g


def pack_cameras(cams, device="cuda") -> torch.Tensor:
    """gsr_camera array on the device, [n_views, 20] 32-bit words.  `cams`
    are objects with fx, fy, cx, cy, R (3x3), t (3), width, height."""
    words = torch.zeros((len(cams), 20), dtype=torch.float32)
    iw = words.view(torch.int32)
    for v, c in enumerate(cams):
        words[v, 0:4] = torch.tensor([c.fx, c.fy, c.cx, c.cy], dtype=torch.float32)
        words[v, 4:13] = torch.as_tensor(c.R, dtype=torch.float32).reshape(9)
        words[v, 13:16] = torch.as_tensor(c.t, dtype=torch.float32).reshape(3)
        iw[v, 16] = int(c.width)
        iw[v, 17] = int(c.height)
    return words.to(device)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _need(t: Optional[torch.Tensor], numel: int, name: str, dtype=None):
    """The kernels index device buffers by the plan's sizes and cannot see a
    tensor's length: reject a buffer that is too small, on the host, or of
    the wrong dtype before its pointer is passed."""
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, the plan needs {numel}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _cams_ptr(cams: torch.Tensor, n_views: int):
    """Pointer to packed cameras (pack_cameras), checked to hold n_views."""
    _need(cams, 20 * n_views, "cams", torch.float32)
    return cams.data_ptr()


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Renderer:
    """One gsr_ctx (device context + plan) and the workspace tensor of its plan."""

    def __init__(self, device: int = 0):
        self.lib = A.load()
        self.device = torch.device("cuda", device)
        ctx = ctypes.c_void_p()
        self._check(self.lib.gsr_create(device, ctypes.byref(ctx)), None)
        self.ctx = ctx
        self.workspace: Optional[torch.Tensor] = None
        self.n = -1
        self.sizes: list = []
        self.capacity = 0
        self.last_generation = 0

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.gsr_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _check(self, status, ctx=True):
        if status != A.GSR_OK:
            msg = self.lib.gsr_last_error(self.ctx).decode() if ctx is not None and getattr(self, "ctx", None) else ""
            base = self.lib.gsr_status_string(status).decode()
            raise GsrError(status, f"{base}: {msg}")

    @property
    def n_views(self) -> int:
        return len(self.sizes)

    @property
    def total_pixels(self) -> int:
        return sum(w * h for w, h in self.sizes)

    def pixel_offsets(self):
        offs, acc = [], 0
        for w, h in self.sizes:
            offs.append(acc)
            acc += w * h
        return offs

    def plan(self, n: int, sizes, pair_capacity: Optional[int] = None, workspace: bool = True) -> int:
        """Plan n Gaussians over views of (width, height) `sizes`; allocates the
        workspace (unless `workspace` is False: for the static-scratch step
        only).  Default capacity: 64 pairs per pixel (at least 1M)."""
        sizes = [(int(w), int(h)) for w, h in sizes]
        if pair_capacity is None:
            pair_capacity = max(1 << 20, 64 * sum(w * h for w, h in sizes))
        wh = (ctypes.c_int32 * (2 * len(sizes)))(*[v for s in sizes for v in s])
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gsr_plan(self.ctx, int(n), len(sizes), wh, int(pair_capacity), ctypes.byref(nbytes)))
        self.workspace = None
        if workspace:
            self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        self.workspace_bytes = int(nbytes.value)
        self.n, self.sizes, self.capacity = int(n), sizes, int(pair_capacity)
        return int(nbytes.value)

    def _ws(self):
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        return aligned, self.workspace.numel() - (aligned - base)

    def ensure_plan(self, n: int, sizes, pair_capacity: Optional[int] = None):
        sizes = [(int(w), int(h)) for w, h in sizes]
        if self.workspace is None or n != self.n or sizes != self.sizes or (
                pair_capacity is not None and pair_capacity > self.capacity):
            self.plan(n, sizes, pair_capacity if pair_capacity is not None else
                      (self.capacity if sizes == self.sizes and self.capacity else None))

    def new_images(self, last=True):
        P = self.total_pixels
        return dict(rgb=torch.empty(3 * P, device=self.device), depth=torch.empty(P, device=self.device),
                    T_final=torch.empty(P, device=self.device),
                    last=torch.empty(P, dtype=torch.int32, device=self.device) if last else None)

    def new_grads(self, n: int, sh: bool = False):
        """Zeroed gradient buffers; with `sh`, d_sh [n, 4, 3] in place of d_rgb."""
        z = lambda *s: torch.zeros(*s, device=self.device)  # noqa: E731
        g = dict(d_mean=z(n, 3), d_log_scale=z(n, 3), d_quat=z(n, 4), d_opacity_logit=z(n),
                 d_rgb=None if sh else z(n, 3), d_pose=z(self.n_views, 6))
        if sh:
            g["d_sh"] = z(n, 4, 3)
        return g

    @staticmethod
    def _images_c(out):
        im = A.gsr_images()
        if out:
            im.rgb, im.depth = _ptr(out.get("rgb")), _ptr(out.get("depth"))
            im.T_final, im.last = _ptr(out.get("T_final")), _ptr(out.get("last"))
            im.loss = _ptr(out.get("loss"))
        return im

    @staticmethod
    def _grads_c(gr, n=0, n_views=0):
        g = A.gsr_grads()
        per = dict(d_mean=3 * n, d_log_scale=3 * n, d_quat=4 * n, d_opacity_logit=n, d_rgb=3 * n, d_pose=6 * n_views,
                   d_sh=12 * n)
        for k in ("d_mean", "d_log_scale", "d_quat", "d_opacity_logit", "d_rgb", "d_pose", "d_sh"):
            _need(gr.get(k), per[k], k, torch.float32)
            setattr(g, k, _ptr(gr.get(k)))
        return g

    def _check_images(self, out):
        P = self.total_pixels
        if out:
            for k, m, dt in (("rgb", 3 * P, torch.float32), ("depth", P, torch.float32),
                             ("T_final", P, torch.float32), ("last", P, torch.int32), ("loss", P, torch.float32)):
                _need(out.get(k), m, k, dt)

    # --------------------------------------------------------- entry points
    def render_forward(self, g: Gaussians, cams: torch.Tensor, cfg: Config, out=None, stream=None, check=True):
        """gsr_render_forward; returns the image dict.  The call itself is
        asynchronous; with `check` the binding then waits for the stream
        (gsr_check_overflow) and, on GSR_E_CAPACITY, grows the pair buffer and
        renders again.  Without it, call check_overflow() later: the outputs
        of an overflowing call are undefined.  The forward's generation goes
        to self.last_generation (render_backward checks it)."""
        out = out if out is not None else self.new_images()
        self._check_images(out)
        gc, cc = g.c(), cfg.to_c()
        for attempt in range(2):
            ws, wsb = self._ws()
            self._check(self.lib.gsr_render_forward(self.ctx, ctypes.byref(gc), _cams_ptr(cams, self.n_views),
                                                    self.n_views, ctypes.byref(cc), ws, wsb,
                                                    ctypes.byref(self._images_c(out)), _stream_ptr(stream)))
            self.last_generation = int(self.lib.gsr_forward_generation(self.ctx))
            if not check:
                break
            try:
                self.check_overflow(stream)
            except GsrError as e:
                if e.status != A.GSR_E_CAPACITY or attempt > 0:
                    raise
                need = int(self.lib.gsr_required_pairs(self.ctx))
                self.plan(self.n, self.sizes, int(need * 1.25) + 1024)
                continue
            break
        return out

    def render_backward(self, g: Gaussians, cams: torch.Tensor, cfg: Config, g_rgb, g_depth, g_T=None,
                        grads=None, stream=None, generation: Optional[int] = None):
        """gsr_render_backward of the forward of `generation` (default: this
        renderer's last forward); GsrError(GSR_E_STATE) when the workspace no
        longer holds that forward's state."""
        grads = grads if grads is not None else self.new_grads(g.n, sh=g.sh is not None)
        P = self.total_pixels
        g_rgb = g_rgb.contiguous()
        g_depth = None if g_depth is None else g_depth.contiguous()
        g_T = None if g_T is None else g_T.contiguous()
        _need(g_rgb, 3 * P, "g_rgb", torch.float32)
        _need(g_depth, P, "g_depth", torch.float32)
        _need(g_T, P, "g_T", torch.float32)
        gen = self.last_generation if generation is None else int(generation)
        gc, cc = g.c(), cfg.to_c()
        ws, wsb = self._ws()
        self._check(self.lib.gsr_render_backward(
            self.ctx, ctypes.byref(gc), _cams_ptr(cams, self.n_views), self.n_views, ctypes.byref(cc), ws, wsb, gen,
            _ptr(g_rgb), _ptr(g_depth), _ptr(g_T), ctypes.byref(self._grads_c(grads, g.n, self.n_views)),
            _stream_ptr(stream)))
        return grads

    def l1_loss_grad(self, rgb, depth, target_rgb, target_depth, pixel_mask=None, w_rgb=1.0, w_depth=0.1,
                     g_rgb=None, g_depth=None, loss=None, loss_cap=None, stream=None):
        g_rgb = g_rgb if g_rgb is not None else torch.empty_like(rgb)
        g_depth = g_depth if g_depth is not None else torch.empty_like(depth)
        loss = loss if loss is not None else torch.zeros(1, device=self.device)
        P = self.total_pixels
        for t, m, name in ((rgb, 3 * P, "rgb"), (depth, P, "depth"), (target_rgb, 3 * P, "target_rgb"),
                           (target_depth, P, "target_depth"), (g_rgb, 3 * P, "g_rgb"), (g_depth, P, "g_depth"),
                           (loss, 1, "loss"), (loss_cap, self.n_views, "loss_cap")):
            _need(t, m, name, torch.float32)
        _need(pixel_mask, P, "pixel_mask", torch.uint8)
        self._check(self.lib.gsr_l1_loss_grad(self.ctx, _ptr(rgb), _ptr(depth), _ptr(target_rgb),
                                              _ptr(target_depth), _ptr(pixel_mask), float(w_rgb), float(w_depth),
                                              _ptr(loss_cap), _ptr(g_rgb), _ptr(g_depth), _ptr(loss),
                                              _stream_ptr(stream)))
        return loss, g_rgb, g_depth

    def loss_median(self, px_loss, pixel_mask=None, factor=10.0, cap_out=None, stream=None):
        """Per view: factor x lower median of px_loss over the pixels with
        pixel_mask != 0 (+inf for a view without such pixels)."""
        cap_out = cap_out if cap_out is not None else torch.empty(self.n_views, device=self.device)
        _need(px_loss, self.total_pixels, "px_loss", torch.float32)
        _need(pixel_mask, self.total_pixels, "pixel_mask", torch.uint8)
        _need(cap_out, self.n_views, "cap_out", torch.float32)
        self._check(self.lib.gsr_loss_median(self.ctx, _ptr(px_loss), _ptr(pixel_mask), float(factor),
                                             _ptr(cap_out), _stream_ptr(stream)))
        return cap_out

    def _fused_args(self, g, cams, cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, out, grads, loss,
                    loss_cap=None):
        ws, wsb = self._ws() if self.workspace is not None else (None, 0)
        P = self.total_pixels
        for t, m, name in ((target_rgb, 3 * P, "target_rgb"), (target_depth, P, "target_depth"), (loss, 1, "loss"),
                           (loss_cap, self.n_views, "loss_cap")):
            _need(t, m, name, torch.float32)
        _need(pixel_mask, P, "pixel_mask", torch.uint8)
        self._check_images(out)
        self._keep = (g.c(), cfg.to_c(), self._images_c(out), self._grads_c(grads, g.n, self.n_views))
        gc, cc, im, gr = self._keep
        return (self.ctx, ctypes.byref(gc), _cams_ptr(cams, self.n_views), self.n_views, ctypes.byref(cc), _ptr(target_rgb),
                _ptr(target_depth), _ptr(pixel_mask), float(w_rgb), float(w_depth), _ptr(loss_cap), ws, wsb,
                ctypes.byref(im) if out else None, ctypes.byref(gr), _ptr(loss))

    def render_l1_fused(self, g: Gaussians, cams, cfg: Config, target_rgb, target_depth, pixel_mask=None,
                        w_rgb=1.0, w_depth=0.1, out=None, grads=None, loss=None, loss_cap=None, stream=None):
        grads = grads if grads is not None else self.new_grads(g.n, sh=g.sh is not None)
        loss = loss if loss is not None else torch.zeros(1, device=self.device)
        args = self._fused_args(g, cams, cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, out, grads, loss,
                                loss_cap)
        self._check(self.lib.gsr_render_l1_fused(*args, _stream_ptr(stream)))
        return loss, grads

    def render_l1_fused_noalloc(self, g: Gaussians, cams, cfg: Config, target_rgb, target_depth, pixel_mask=None,
                                w_rgb=1.0, w_depth=0.1, out=None, grads=None, loss=None, loss_cap=None, stream=None):
        """gsr_render_l1_fused_noalloc: the fused step on the library's static
        scratch (the plan must fit A.GSR_NOALLOC_SCRATCH_BYTES); `grads` and
        `loss` are caller buffers, as for render_l1_fused."""
        grads = grads if grads is not None else self.new_grads(g.n, sh=g.sh is not None)
        loss = loss if loss is not None else torch.zeros(1, device=self.device)
        args = self._fused_args(g, cams, cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, out, grads, loss,
                                loss_cap)
        args = args[:11] + args[13:]  # no workspace pointer and size
        self._check(self.lib.gsr_render_l1_fused_noalloc(*args, _stream_ptr(stream)))
        return loss, grads

    def check_overflow_noalloc(self, stream=None):
        """gsr_check_overflow on the static scratch (NULL workspace)."""
        self._check(self.lib.gsr_check_overflow(self.ctx, None, _stream_ptr(stream)))

    def graph_capture(self, g, cams, cfg, target_rgb, target_depth, pixel_mask=None, w_rgb=1.0, w_depth=0.1,
                      out=None, grads=None, loss=None, loss_cap=None, stream=None):
        """Capture the fused step into a HIP graph (torch.cuda stream required)."""
        args = self._fused_args(g, cams, cfg, target_rgb, target_depth, pixel_mask, w_rgb, w_depth, out, grads, loss,
                                loss_cap)
        s = stream if stream is not None else torch.cuda.current_stream()
        if s.cuda_stream == 0:
            raise ValueError("graph capture needs a non-default stream")
        self._check(self.lib.gsr_graph_capture(*args, s.cuda_stream))

    def graph_launch(self, stream=None):
        self._check(self.lib.gsr_graph_launch(self.ctx, _stream_ptr(stream)))

    def check_overflow(self, stream=None):
        ws, _ = self._ws()
        self._check(self.lib.gsr_check_overflow(self.ctx, ws, _stream_ptr(stream)))

    def required_pairs(self) -> int:
        return int(self.lib.gsr_required_pairs(self.ctx))

    def pair_count(self, stream=None) -> int:
        ws, _ = self._ws()
        return int(self.lib.gsr_pair_count(self.ctx, ws, _stream_ptr(stream)))

    def debug_tiles(self):
        """(tile_ranges [T,2] int32, sorted_ids [pairs] int64) copied to the host."""
        ws, _ = self._ws()
        r, ids, tt = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        self._check(self.lib.gsr_debug_tiles(self.ctx, ws, ctypes.byref(r), ctypes.byref(ids), ctypes.byref(tt)))
        torch.cuda.current_stream().synchronize()
        base = self.workspace.data_ptr()
        T = int(tt.value)
        ro = r.value - base
        rng = self.workspace[ro:ro + 8 * T].view(torch.int32).reshape(T, 2).cpu()
        npairs = self.pair_count()
        io = ids.value - base
        sid = self.workspace[io:io + 4 * npairs].view(torch.int32).cpu().to(torch.int64) & 0xFFFFFFFF
        return rng, sid

    def get_tuning(self) -> dict:
        t = A.gsr_tuning()
        self._check(self.lib.gsr_get_tuning(self.ctx, ctypes.byref(t)))
        return dict(blocks_per_cu=t.blocks_per_cu, tiles_per_pop=t.tiles_per_pop, lpt_order=t.lpt_order,
                    batch=t.batch)

    def set_tuning(self, blocks_per_cu=4, tiles_per_pop=1, lpt_order=1, batch=192):
        t = A.gsr_tuning(blocks_per_cu, tiles_per_pop, lpt_order, batch)
        self._check(self.lib.gsr_set_tuning(self.ctx, ctypes.byref(t)))

    def autotune(self, g, cams, cfg, target_rgb, target_depth, pixel_mask=None, w_rgb=1.0, w_depth=0.1,
                 reps=3, stream=None) -> dict:
        grads = self.new_grads(g.n, sh=g.sh is not None)
        loss = torch.zeros(1, device=self.device)
        ws, wsb = self._ws()
        P = self.total_pixels
        _need(target_rgb, 3 * P, "target_rgb", torch.float32)
        _need(target_depth, P, "target_depth", torch.float32)
        _need(pixel_mask, P, "pixel_mask", torch.uint8)
        gc, cc, gr = g.c(), cfg.to_c(), self._grads_c(grads, g.n, self.n_views)
        best = A.gsr_tuning()
        self._check(self.lib.gsr_autotune(self.ctx, ctypes.byref(gc), _cams_ptr(cams, self.n_views), self.n_views,
                                          ctypes.byref(cc), _ptr(target_rgb), _ptr(target_depth), _ptr(pixel_mask),
                                          float(w_rgb), float(w_depth), ws, wsb, ctypes.byref(gr), _ptr(loss),
                                          int(reps), ctypes.byref(best), _stream_ptr(stream)))
        return dict(blocks_per_cu=best.blocks_per_cu, tiles_per_pop=best.tiles_per_pop, lpt_order=best.lpt_order,
                    batch=best.batch)


    def select_reliable(self, g: Gaussians, cam: torch.Tensor, depth_obs: torch.Tensor, width: int, height: int,
                        eps: float, z_near: float = 0.2, mask_out: Optional[torch.Tensor] = None, stream=None):
        """gsr_select_reliable: uint8 mask of the Gaussians kept for the fine
        tracking stage (Eq. 12).  `cam` is one packed camera (the coarse pose)."""
        out = mask_out if mask_out is not None else torch.empty(g.n, dtype=torch.uint8, device=self.device)
        _need(depth_obs, int(width) * int(height), "depth_obs", torch.float32)
        _need(out, g.n, "mask_out", torch.uint8)
        gc = g.c()
        self._check(self.lib.gsr_select_reliable(self.ctx, ctypes.byref(gc), _cams_ptr(cam, 1), depth_obs.data_ptr(),
                                                 int(width), int(height), float(eps), float(z_near), out.data_ptr(),
                                                 _stream_ptr(stream)))
        return out

    # ------------------------------------------------------------ poses
    def expand_add(self, cams: torch.Tensor, T_final, depth, depth_obs, rgb_obs, out: dict, n: int, capacity: int,
                   tau_T: float, tau_D: float, scale_factor: float = 1.0, opacity_logit_init: float = -2.1972246,
                   pixel_flag: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None, stream=None):
        """gsr_expand_add over the planned views (Eq. 8): appends a Gaussian
        per unreliable pixel to the arrays of `out` (keys mean, log_scale,
        quat, opacity_logit and rgb and/or sh (a spherical-harmonic map,
        [capacity, 4, 3]); `capacity` rows) from row n on.  Returns the device
        int64 count of unreliable pixels.  The default initial opacity logit
        is that of opacity 0.1."""
        P = self.total_pixels
        for t, m, name in ((T_final, P, "T_final"), (depth, P, "depth"), (depth_obs, P, "depth_obs"),
                           (rgb_obs, 3 * P, "rgb_obs")):
            _need(t, m, name, torch.float32)
        _need(pixel_flag, P, "pixel_flag", torch.uint8)
        per = dict(mean=3, log_scale=3, quat=4, opacity_logit=1, rgb=3, sh=12)
        if int(capacity) > int(n) and out.get("rgb") is None and out.get("sh") is None:
            raise ValueError("expand_add: out needs rgb or sh")
        o = A.gsr_gaussians_out()
        for k, c in per.items():
            if k in ("rgb", "sh") and out.get(k) is None:
                continue
            _need(out.get(k), c * int(capacity), k, torch.float32)
            setattr(o, k, _ptr(out.get(k)))
        count = count if count is not None else torch.zeros(1, dtype=torch.int64, device=self.device)
        _need(count, 1, "count", torch.int64)
        prm = A.gsr_expand_params(float(tau_T), float(tau_D), float(scale_factor), float(opacity_logit_init))
        ws, wsb = self._ws()
        self._check(self.lib.gsr_expand_add(self.ctx, _cams_ptr(cams, self.n_views), self.n_views, _ptr(T_final),
                                            _ptr(depth), _ptr(depth_obs), _ptr(rgb_obs), ctypes.byref(prm), ws, wsb,
                                            int(n), int(capacity), ctypes.byref(o), _ptr(pixel_flag), _ptr(count),
                                            _stream_ptr(stream)))
        return count

    def expand_delete(self, g: Gaussians, cam: torch.Tensor, depth_obs: torch.Tensor, width: int, height: int,
                      gamma: float, eta: float, z_near: float = 0.2, logit_out: Optional[torch.Tensor] = None,
                      decayed: Optional[torch.Tensor] = None, stream=None):
        """gsr_expand_delete (Eq. 9) for one view; returns (new logits,
        decayed mask).  logit_out may be g's own opacity-logit tensor."""
        logit_out = logit_out if logit_out is not None else torch.empty(g.n, device=self.device)
        decayed = decayed if decayed is not None else torch.empty(g.n, dtype=torch.uint8, device=self.device)
        _need(logit_out, g.n, "logit_out", torch.float32)
        _need(decayed, g.n, "decayed", torch.uint8)
        _need(depth_obs, int(width) * int(height), "depth_obs", torch.float32)
        gc = g.c()
        self._check(self.lib.gsr_expand_delete(self.ctx, ctypes.byref(gc), _cams_ptr(cam, 1), _ptr(depth_obs),
                                               int(width), int(height), float(gamma), float(eta), float(z_near),
                                               _ptr(logit_out), _ptr(decayed), _stream_ptr(stream)))
        return logit_out, decayed

    def pose_apply(self, xi: torch.Tensor, cams_in: torch.Tensor, cams_out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
        """gsr_pose_apply: cameras with the poses Exp(xi_v) T_v ([V, 6] float32 xi)."""
        V = int(cams_in.shape[0])
        out = cams_out if cams_out is not None else torch.empty_like(cams_in)
        _need(xi.contiguous(), 6 * V, "xi", torch.float32)
        _need(out, 20 * V, "cams_out", torch.float32)
        xi = xi.contiguous()
        self._check(self.lib.gsr_pose_apply(self.ctx, V, xi.data_ptr(), _cams_ptr(cams_in, V), out.data_ptr(),
                                            _stream_ptr(stream)))
        return out

    def pose_xi_grad(self, xi: torch.Tensor, d_pose: torch.Tensor, stream=None) -> torch.Tensor:
        """gsr_pose_xi_grad: J_l(xi)^T d_pose per view."""
        V = int(d_pose.shape[0])
        xi, d_pose = xi.contiguous(), d_pose.contiguous()
        _need(xi, 6 * V, "xi", torch.float32)
        _need(d_pose, 6 * V, "d_pose", torch.float32)
        out = torch.empty(V, 6, device=self.device)
        self._check(self.lib.gsr_pose_xi_grad(self.ctx, V, xi.data_ptr(), d_pose.data_ptr(), out.data_ptr(),
                                              _stream_ptr(stream)))
        return out

    def pose_from_qt(self, q: torch.Tensor, t: torch.Tensor, cams_in: torch.Tensor,
                     cams_out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """gsr_pose_from_qt: cameras with R = R(q / |q|) and t ([V, 4], [V, 3])."""
        V = int(cams_in.shape[0])
        q, t = q.contiguous(), t.contiguous()
        _need(q, 4 * V, "q", torch.float32)
        _need(t, 3 * V, "t", torch.float32)
        out = cams_out if cams_out is not None else torch.empty_like(cams_in)
        _need(out, 20 * V, "cams_out", torch.float32)
        self._check(self.lib.gsr_pose_from_qt(self.ctx, V, q.data_ptr(), t.data_ptr(), _cams_ptr(cams_in, V),
                                              out.data_ptr(), _stream_ptr(stream)))
        return out

    def pose_qt_grad(self, q: torch.Tensor, t: torch.Tensor, d_pose: torch.Tensor, stream=None):
        """gsr_pose_qt_grad: (d_q [V, 4], d_t [V, 3]) from the left-perturbation gradient."""
        V = int(d_pose.shape[0])
        q, t, d_pose = q.contiguous(), t.contiguous(), d_pose.contiguous()
        _need(q, 4 * V, "q", torch.float32)
        _need(t, 3 * V, "t", torch.float32)
        _need(d_pose, 6 * V, "d_pose", torch.float32)
        d_q = torch.empty(V, 4, device=self.device)
        d_t = torch.empty(V, 3, device=self.device)
        self._check(self.lib.gsr_pose_qt_grad(self.ctx, V, q.data_ptr(), t.data_ptr(), d_pose.data_ptr(),
                                              d_q.data_ptr(), d_t.data_ptr(), _stream_ptr(stream)))
        return d_q, d_t

    # ------------------------------------------------------------ profiling
    def set_profiling(self, enable: bool = True):
        self._check(self.lib.gsr_set_profiling(self.ctx, 1 if enable else 0))

    def stage_times(self) -> dict:
        """Summed milliseconds per stage since the last query, and the call count."""
        ms = (ctypes.c_double * len(A.STAGES))()
        calls = ctypes.c_int64()
        self._check(self.lib.gsr_stage_times(self.ctx, ms, ctypes.byref(calls)))
        out = {k: float(ms[i]) for i, k in enumerate(A.STAGES)}
        out["calls"] = int(calls.value)
        return out

    def work_counts(self, g: Gaussians, cfg: Config, stream=None) -> dict:
        """Work of the last forward or fused call, which used `g` and `cfg`."""
        ws, _ = self._ws()
        out = (ctypes.c_int64 * 4)()
        gc, cc = g.c(), cfg.to_c()
        self._check(self.lib.gsr_work_counts(self.ctx, ctypes.byref(gc), ctypes.byref(cc), ws, _stream_ptr(stream),
                                             out))
        return dict(pairs=int(out[0]), fwd_evals=int(out[1]), blended=int(out[2]), bwd_evals=int(out[3]))


# ------------------------------------------------------------------ autograd

class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, rgb, pose_xi, renderer, cams0, cfg, mask, check):
        sh_mode = rgb.dim() == 3  # [n, 4, 3]: spherical-harmonic colour
        g = Gaussians(mean.contiguous(), log_scale.contiguous(), quat.contiguous(), opacity_logit.contiguous(),
                      None if sh_mode else rgb.contiguous(), mask, rgb.contiguous() if sh_mode else None)
        xi = pose_xi.detach().to(torch.float32).contiguous()
        cams = renderer.pose_apply(xi, cams0)  # T = Exp(xi) T0 on the device
        out = renderer.render_forward(g, cams, cfg, check=check)
        ctx.renderer, ctx.cams, ctx.cfg, ctx.g, ctx.xi = renderer, cams, cfg, g, xi
        ctx.generation = renderer.last_generation
        ctx.mark_non_differentiable(out["last"])
        return out["rgb"], out["depth"], out["T_final"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_T):
        r, g = ctx.renderer, ctx.g
        P = r.total_pixels
        dev = r.device
        g_rgb = torch.zeros(3 * P, device=dev) if g_rgb is None else g_rgb.contiguous()
        g_depth = torch.zeros(P, device=dev) if g_depth is None else g_depth.contiguous()
        g_T = None if g_T is None else g_T.contiguous()
        grads = r.render_backward(g, ctx.cams, ctx.cfg, g_rgb, g_depth, g_T, generation=ctx.generation)
        d_xi = r.pose_xi_grad(ctx.xi, grads["d_pose"])
        d_col = grads["d_sh"] if g.sh is not None else grads["d_rgb"]
        return (grads["d_mean"], grads["d_log_scale"], grads["d_quat"], grads["d_opacity_logit"], d_col,
                d_xi, None, None, None, None, None)


def render(renderer: Renderer, mean, log_scale, quat, opacity_logit, rgb, cams: torch.Tensor,
           cfg: Optional[Config] = None, pose_xi: Optional[torch.Tensor] = None, mask=None, check: bool = True):
    """Differentiable render of every planned view at the poses
    T_v = Exp(xi_v) T0_v, T0_v the pose of cams[v] and xi_v = pose_xi[v]
    (zero when pose_xi is None).  `rgb` is [n, 3] RGB or [n, 4, 3] degree-1
    spherical-harmonic coefficients (view-dependent colour).  Returns flat (rgb, depth, T_final) over the
    concatenated views; the gradient of pose_xi is J_l(xi)^T times the
    renderer's left-perturbation pose gradient (gsr_pose_xi_grad).  The
    backward of a call must run before the renderer renders again (each
    forward's state lives in the renderer's one workspace; a later forward
    makes an earlier call's backward raise GsrError(GSR_E_STATE)).  With
    check=False the forward does not wait for the stream: call
    renderer.check_overflow() before trusting the outputs."""
    cfg = cfg or Config()
    if pose_xi is None:
        pose_xi = torch.zeros(renderer.n_views, 6, device=renderer.device)
    return _RenderFn.apply(mean, log_scale, quat, opacity_logit, rgb, pose_xi, renderer, cams, cfg, mask, check)


def split_views(flat: torch.Tensor, sizes, channels: int = 1):
    """Split a concatenated image buffer into per-view [C, H, W] (or [H, W])."""
    out, off = [], 0
    for w, h in sizes:
        k = channels * w * h
        x = flat[off:off + k]
        out.append(x.reshape(channels, h, w) if channels > 1 else x.reshape(h, w))
        off += k
    return out
