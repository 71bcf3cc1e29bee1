"""Full-size checks of the two many-view workloads, in the launch
configuration bench.py times (one graph-captured fused step over all views,
gradients and loss overwritten by the step; here it also writes the images):

- 16 keyframes of mixed resolution (4x320x240, 8x640x480, 4x1200x680) over
  1M Gaussians, gradients to every Gaussian parameter and every pose;
- 72 pose hypotheses (64 at 600x340, 8 at 1200x680) over 500k Gaussians,
  pose gradients only.

For sampled views (one or more of each resolution): every tile's list length
and sampled tiles' lists bit-exact against the oracle, and sampled tiles'
pixels within 1e-4.  For all views: the batched step's loss and gradients
equal those of one fused call per view (same kernels per view; only the
order of the floating-point additions across views differs)."""
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


def _captured_step(gsr, r, g, cams_d, cfg, t_rgb, t_d, grads):
    """Capture the fused step into a graph, replay it twice (the second
    replay overwrites the first's gradients and loss) and return the images
    and the loss."""
    out = r.new_images()
    loss = torch.zeros(1, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, out=out, grads=grads, loss=loss, stream=s)
    s.synchronize()
    for _ in range(2):
        r.graph_launch(stream=s)
    s.synchronize()
    r.check_overflow(stream=s)
    return out, loss


def _check_view(lists, out, scene, cams, sizes, v, n_tiles=12, n_px_tiles=4):
    """View v's tile lists (every list length, sampled lists; `lists` = the
    renderer's debug_tiles) bit-exact and sampled tiles' pixels within 1e-4
    of the oracle."""
    cam = cams[v]
    proj = O.project(scene, cam, O.Config().as_f32())
    assert not proj["bin_ambiguous"].any()
    starts, gauss = O.tile_lists(proj)
    off = sum(((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes[:v])
    T = proj["TX"] * proj["TY"]
    rng, sid = lists
    lens = rng[off:off + T, 1] - rng[off:off + T, 0]
    for t in np.nonzero(lens != np.diff(starts))[0]:
        a, b = rng[off + t]
        got_t, want_t = set((sid[a:b] - v * scene.n).tolist()), set(gauss[starts[t]:starts[t + 1]].tolist())
        for i in sorted(got_t ^ want_t):
            print(f"view {v} tile {t}: Gaussian {i} {'only on the GPU' if i in got_t else 'only in the oracle'}; "
                  f"uv {proj['uv'][i]} conic {proj['conic'][i]} opacity {proj['opacity'][i]} rect {proj['rect'][i]} "
                  f"z {proj['z'][i]}", flush=True)
    np.testing.assert_array_equal(lens, np.diff(starts))
    sel = np.random.default_rng(v).choice(T, n_tiles, replace=False)
    for t in sel:
        a, b = rng[off + t]
        np.testing.assert_array_equal(sid[a:b] - v * scene.n, gauss[starts[t]:starts[t + 1]])
    tiles = sorted(int(t) for t in sel[:n_px_tiles])
    o = O.render(scene, cam, O.Config(), tiles=tiles, proj=proj, lists=(starts, gauss))
    got = H.split_images(out, sizes)[v]
    H.assert_images_close(got, o, done=o["done"], max_ambiguous=0.03)


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
