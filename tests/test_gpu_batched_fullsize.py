"""Full-size checks of the two many-view workloads, in the launch
configuration bench.py times (one graph-captured fused step over all views,
gradients and loss overwritten by the step; here it also writes the images):

- 16 keyframes of mixed resolution (4x320x240, 8x640x480, 4x1200x680) over
  1M Gaussians, gradients to every Gaussian parameter and every pose;
- 72 pose hypotheses (64 at 600x340, 8 at 1200x680) over 500k Gaussians,
  pose gradients only.

For sampled views (one or more of each resolution): every tile's list no
longer than the oracle's, sampled tiles' lists in-order subsequences of the
oracle's that keep every Gaussian reaching alpha_min in the tile, and
sampled tiles' pixels within 1e-4.  For all views: the batched step's loss
and gradients equal those of one fused call per view (same kernels per view;
only the order of the floating-point additions across views differs).  And
against the FP64 oracle: with the loss restricted to 20 sampled tiles of
three views of each resolution, every Gaussian's gradient and those views'
poses within 1e-3."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _targets(gsr, r, g, cams_d):
    """Targets as the benchmark makes them: the scene's own render plus 5%
    noise (depth 0 where the accumulated opacity is below 0.5)."""
    out = r.render_forward(g, cams_d, gsr.Config())
    torch.cuda.synchronize()
    t_rgb, t_d = W.noisy_targets(out["rgb"].cpu().numpy(), out["depth"].cpu().numpy(), seed=1, sigma=0.05,
                                 min_alpha=0.5, alpha=1.0 - out["T_final"].cpu().numpy())
    return H.to_dev(t_rgb), H.to_dev(t_d)


def _captured_step(gsr, r, g, cams_d, cfg, t_rgb, t_d, grads, mask=None):
    """Capture the fused step into a graph, replay it twice (the second
    replay overwrites the first's gradients and loss) and return the images
    and the loss."""
    out = r.new_images()
    loss = torch.zeros(1, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r.graph_capture(g, cams_d, cfg, t_rgb, t_d, mask, 1.0, 0.1, out=out, grads=grads, loss=loss, stream=s)
    s.synchronize()
    for _ in range(2):
        r.graph_launch(stream=s)
    s.synchronize()
    r.check_overflow(stream=s)
    return out, loss


def _check_view(lists, out, scene, cams, sizes, v, n_tiles=12, n_px_tiles=4):
    """View v's tile lists (every list no longer than the oracle's; sampled
    lists checked in full against it; `lists` = the renderer's debug_tiles)
    and sampled tiles' pixels within 1e-4 of the oracle."""
    cam = cams[v]
    proj = O.project(scene, cam, O.Config().as_f32())
    assert not proj["bin_ambiguous"].any()
    olists = O.tile_lists(proj)
    off = sum(((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes[:v])
    T = proj["TX"] * proj["TY"]
    rng, sid = lists
    assert np.all(rng[off:off + T, 1] - rng[off:off + T, 0] <= np.diff(olists[0]))
    sel = np.random.default_rng(v).choice(T, n_tiles, replace=False)
    H.check_view_lists(rng, sid, off, v * scene.n, proj, olists, cam.width, cam.height, O.Config(), tiles=sel)
    tiles = sorted(int(t) for t in sel[:n_px_tiles])
    o = O.render(scene, cam, O.Config(), tiles=tiles, proj=proj, lists=olists)
    got = H.split_images(out, sizes)[v]
    H.assert_images_close(got, o, done=o["done"], max_ambiguous=0.01, gpu_lists=(rng, sid, off, v * scene.n))
    return proj, olists


def _loss_rtol(sizes):
    """The loss is a float32 sum of one partial per tile, added by atomics in
    whatever order the tiles finish (and per view in the separate calls):
    two such sums differ by about sqrt(tiles) float32 roundings of the total;
    six times that bounds them."""
    tiles = sum(((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes)
    return 6.0 * np.sqrt(tiles) * 2.0 ** -24


def _per_view_calls(gsr, g, cams, sizes, cfg_acc, t_rgb, t_d, grads):
    """One fused call per view, adding into the same gradients and loss (one
    renderer per resolution, reused view after view)."""
    rs = {}
    for w, h in set(sizes):
        rs[(w, h)] = gsr.Renderer()
        rs[(w, h)].plan(g.n, [(w, h)])
    loss = torch.zeros(1, device="cuda")
    gr1 = dict(grads)
    po = 0
    for v, (w, h) in enumerate(sizes):
        gr1["d_pose"] = grads["d_pose"][v:v + 1]
        rs[(w, h)].render_l1_fused(g, gsr.pack_cameras([cams[v]]), cfg_acc, t_rgb[3 * po:3 * (po + w * h)],
                                   t_d[po:po + w * h], None, 1.0, 0.1, grads=gr1, loss=loss)
        po += w * h
    torch.cuda.synchronize()
    for r in rs.values():
        r.check_overflow()
    return loss


def _oracle_gradient_parity(gsr, r, g, scene, cams, sizes, views, cfg, t_rgb, t_d, grads, gauss_grads,
                            n_tiles=20):
    """The captured step with its loss restricted (pixel_mask) to n_tiles
    sampled tiles of each of `views`: every Gaussian's gradient (when
    gauss_grads) and those views' poses against the FP64 oracle at 1e-3,
    all other poses exactly zero.  The backward is linear in the per-pixel
    upstream gradient, so the oracle over the sampled tiles is the whole
    answer.  Pixels whose loss sign or threshold decisions are ambiguous in
    float32 are masked on both sides."""
    P = sum(w * h for w, h in sizes)
    mask = np.zeros(P, np.uint8)
    offs = np.cumsum([0] + [w * h for w, h in sizes])
    trgb = t_rgb.cpu().numpy()
    tdep = t_d.cpu().numpy()
    ocfg = O.Config().as_f32()
    per_view = {}
    for v in views:
        cam = cams[v]
        w, h = sizes[v]
        proj = O.project(scene, cam, ocfg)
        lists = O.tile_lists(proj)
        T = proj["TX"] * proj["TY"]
        tiles = sorted(np.random.default_rng(100 + v).choice(T, n_tiles, replace=False).tolist())
        fwd = O.render(scene, cam, ocfg, tiles=tiles, proj=proj, lists=lists)
        po = offs[v]
        tr = trgb[3 * po:3 * (po + w * h)].reshape(3, h, w)
        td = tdep[po:po + w * h].reshape(h, w)
        m = fwd["done"] & ~fwd["ambiguous_grad"]
        m &= ~(np.abs(fwd["rgb"] - tr) < 1e-4).any(axis=0) & ~(np.abs(fwd["depth"] - td) < 1e-4)
        mask[po:po + w * h] = m.reshape(-1)
        per_view[v] = (proj, lists, tiles, fwd, tr, td, m)
        print(f"oracle view {v} {sizes[v]}: {int(m.sum())} px in {len(tiles)} tiles", flush=True)
    _captured_step(gsr, r, g, gsr.pack_cameras(cams), cfg, t_rgb, t_d, grads, mask=H.to_dev(mask, torch.uint8))
    got = {k: t.cpu().numpy() for k, t in grads.items()}
    ref, g2_any = None, np.zeros(scene.n, bool)
    names = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
    for v, (proj, lists, tiles, fwd, tr, td, m) in per_view.items():
        _, gC, gD = O.l1_loss(fwd["rgb"], fwd["depth"], tr, td, m, 1.0, 0.1)
        g2, _ = O.backward_2d(scene, cams[v], ocfg, gC, gD, None, fwd=fwd, tiles=tiles)
        nz = np.nonzero(np.abs(g2).sum(1) > 0)[0]
        g2_any[nz] = True
        # The chain is per Gaussian (a Gaussian without a 2D gradient adds
        # nothing, also to the pose): run it on the ones with a gradient.
        sub = {k: (a[nz] if isinstance(a, np.ndarray) and a.ndim >= 1 and a.shape[0] == scene.n else a)
               for k, a in proj.items()}
        sub["n"] = nz.size
        bs = O.backward_params(sub, g2[nz], ocfg)
        b = {"pose": bs["pose"]}
        for k in names:
            b[k] = np.zeros((scene.n,) + bs[k].shape[1:])
            b[k][nz] = bs[k]
        assert H.rel_err(got["d_pose"][v], b["pose"]) <= 1e-3, (v, got["d_pose"][v], b["pose"])
        if gauss_grads:
            ref = {k: b[k] for k in names} if ref is None else {k: ref[k] + b[k] for k in names}
        del proj, lists
    others = [v for v in range(len(cams)) if v not in per_view]
    assert not np.any(got["d_pose"][others])
    if gauss_grads:
        sel = np.nonzero(g2_any)[0]
        rest = np.nonzero(~g2_any)[0]
        print(f"Gaussians with a gradient: {sel.size}", flush=True)
        assert sel.size >= 100
        for k in names:
            assert not np.any(got["d_" + k][rest]), k
        H.assert_grads_close({k: got["d_" + k][sel] for k in names}, {k: ref[k][sel] for k in names})


def test_sixteen_keyframes_one_launch(gsr_lib):
    gsr = gsr_lib
    scene = W.room_scene(1_000_000, seed=0)
    cams = W.mapping_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    print("CASE 16 keyframes, 1M Gaussians, captured fused step", flush=True)
    g = H.gpu_scene(gsr, scene)
    cams_d = gsr.pack_cameras(cams)
    r = gsr.Renderer()
    r.plan(scene.n, sizes)
    t_rgb, t_d = _targets(gsr, r, g, cams_d)
    r.plan(scene.n, sizes, pair_capacity=int(r.pair_count() * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    grads = r.new_grads(scene.n)
    out, loss = _captured_step(gsr, r, g, cams_d, cfg, t_rgb, t_d, grads)
    lists = tuple(x.numpy() for x in r.debug_tiles())
    for v in (0, 4, 13):  # 320x240, 640x480, 1200x680
        print(f"CASE keyframe {v} {sizes[v]} against the oracle", flush=True)
        _check_view(lists, out, scene, cams, sizes, v)
    del lists
    got = {k: t.cpu().numpy() for k, t in grads.items()}
    print("CASE 16 per-keyframe fused calls", flush=True)
    ref = {k: torch.zeros_like(t) for k, t in grads.items()}
    loss_ref = _per_view_calls(gsr, g, cams, sizes, gsr.Config(), t_rgb, t_d, ref)
    assert abs(loss.item() - loss_ref.item()) <= _loss_rtol(sizes) * loss_ref.item(), (loss.item(), loss_ref.item())
    for k in ref:
        H.assert_close_scaled(got[k], ref[k].cpu().numpy(), what=k)


def test_pose_hypotheses_one_launch(gsr_lib):
    gsr = gsr_lib
    scene = W.room_scene(500_000, seed=0)
    cams = W.hypothesis_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    print("CASE 72 pose hypotheses, 500k Gaussians, captured fused step (pose gradients)", flush=True)
    g = H.gpu_scene(gsr, scene)
    # Targets rendered from the unperturbed pose at each resolution.
    base_full = W.camera_replica()
    h = W.camera_hyp_half()
    base_half = base_full.with_size(h.fx, h.fy, h.cx, h.cy, h.width, h.height)
    tg = {}
    for cam in (base_half, base_full):
        rt = gsr.Renderer()
        rt.plan(scene.n, [(cam.width, cam.height)])
        tg[(cam.width, cam.height)] = _targets(gsr, rt, g, gsr.pack_cameras([cam]))
        del rt
    t_rgb = torch.cat([tg[s][0] for s in sizes])
    t_d = torch.cat([tg[s][1] for s in sizes])
    cams_d = gsr.pack_cameras(cams)
    r = gsr.Renderer()
    r.plan(scene.n, sizes)
    r.render_forward(g, cams_d, gsr.Config())
    r.plan(scene.n, sizes, pair_capacity=int(r.pair_count() * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    grads = {"d_pose": torch.zeros(len(cams), 6, device="cuda")}
    out, loss = _captured_step(gsr, r, g, cams_d, cfg, t_rgb, t_d, grads)
    lists = tuple(x.numpy() for x in r.debug_tiles())
    for v in (0, 63, 71):  # 600x340, 600x340, 1200x680
        print(f"CASE hypothesis {v} {sizes[v]} against the oracle", flush=True)
        _check_view(lists, out, scene, cams, sizes, v)
    del lists
    got = grads["d_pose"].cpu().numpy()
    print("CASE 72 per-pose fused calls", flush=True)
    ref = {"d_pose": torch.zeros(len(cams), 6, device="cuda")}
    loss_ref = _per_view_calls(gsr, g, cams, sizes, gsr.Config(flags=gsr.GSR_POSE_GRAD), t_rgb, t_d, ref)
    assert abs(loss.item() - loss_ref.item()) <= _loss_rtol(sizes) * loss_ref.item(), (loss.item(), loss_ref.item())
    want = ref["d_pose"].cpu().numpy()
    assert np.abs(want).max() > 0
    for v in range(len(cams)):
        H.assert_close_scaled(got[v], want[v], what=("pose", v))


def test_sixteen_keyframes_oracle_gradients(gsr_lib):
    gsr = gsr_lib
    scene = W.room_scene(1_000_000, seed=0)
    cams = W.mapping_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    print("CASE 16 keyframes, 1M Gaussians: oracle gradients over sampled tiles", flush=True)
    g = H.gpu_scene(gsr, scene)
    r = gsr.Renderer()
    r.plan(scene.n, sizes)
    t_rgb, t_d = _targets(gsr, r, g, gsr.pack_cameras(cams))
    r.plan(scene.n, sizes, pair_capacity=int(r.pair_count() * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    # three views of each resolution (320x240: 0-3, 640x480: 4-11, 1200x680: 12-15)
    _oracle_gradient_parity(gsr, r, g, scene, cams, sizes, (0, 2, 3, 4, 7, 11, 12, 13, 15), cfg, t_rgb, t_d,
                            r.new_grads(scene.n), True)


def test_pose_hypotheses_oracle_gradients(gsr_lib):
    gsr = gsr_lib
    scene = W.room_scene(500_000, seed=0)
    cams = W.hypothesis_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    print("CASE 72 pose hypotheses, 500k Gaussians: oracle pose gradients over sampled tiles", flush=True)
    g = H.gpu_scene(gsr, scene)
    r = gsr.Renderer()
    r.plan(scene.n, sizes)
    t_rgb, t_d = _targets(gsr, r, g, gsr.pack_cameras(cams))  # noisy renders of the hypotheses themselves
    r.plan(scene.n, sizes, pair_capacity=int(r.pair_count() * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    # three views of each resolution (600x340: 0-63, 1200x680: 64-71)
    _oracle_gradient_parity(gsr, r, g, scene, cams, sizes, (0, 31, 63, 64, 68, 71), cfg, t_rgb, t_d,
                            {"d_pose": torch.zeros(len(cams), 6, device="cuda")}, False)
