"""Full-size checks at the benchmark's workload (300k Gaussians, 1200x680) and
in the launch configuration bench.py times (graph-captured fused step):
the pair count equal to the oracle's, every tile list checked against the
oracle's, sampled tiles' pixels within 1e-4, exact FP64 gradients of every
Gaussian with the upstream gradient restricted to sampled tiles, and
properties of the backward that hold at any size (translation gauge
identity, colour-gradient sum, linearity, fused step equal to forward + L1
+ backward)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2(gsr_lib):
    gsr = gsr_lib
    scene, cam = W.room_scene(300_000, seed=0), W.camera_replica()
    print("CASE full-size 300k 1200x680", flush=True)
    r = gsr.Renderer()
    r.plan(scene.n, [(cam.width, cam.height)])
    g = H.gpu_scene(gsr, scene)
    cams_d = gsr.pack_cameras([cam])
    out = r.render_forward(g, cams_d, gsr.Config())
    torch.cuda.synchronize()
    proj = O.project(scene, cam, O.Config().as_f32())
    lists = O.tile_lists(proj)
    return dict(gsr=gsr, scene=scene, cam=cam, r=r, g=g, cams_d=cams_d, out=out, proj=proj, lists=lists)


def test_pairs_and_lists_match_oracle(c2):
    """Pair count equal to the oracle's (every tile of every 3-sigma
    rectangle), and every tile's list an in-order subsequence of the
    oracle's that keeps each Gaussian reaching alpha_min at a pixel of the
    tile (all 3 225 tiles, every pixel evaluated in FP64)."""
    r, proj, lists, cam = c2["r"], c2["proj"], c2["lists"], c2["cam"]
    assert not proj["bin_ambiguous"].any()
    assert r.pair_count() == H.rect_pairs(proj)
    rng, sid = r.debug_tiles()
    rng, sid = rng.numpy(), sid.numpy()
    n_or, n_gpu, n_amb = H.check_view_lists(rng, sid, 0, 0, proj, lists, cam.width, cam.height, O.Config())
    print(f"oracle pairs {n_or}, listed {n_gpu}, ambiguous drops {n_amb}", flush=True)
    assert n_or == H.rect_pairs(proj) and n_gpu < n_or


def test_sampled_tiles_match_oracle(c2):
    proj, cam = c2["proj"], c2["cam"]
    T = proj["TX"] * proj["TY"]
    sample = list(np.random.default_rng(1).choice(T, 12, replace=False)) + [T - 1]
    o = O.render(c2["scene"], cam, O.Config(), tiles=sample, proj=proj, lists=c2["lists"])
    g = H.split_images(c2["out"], [(cam.width, cam.height)])[0]
    rng, sid = c2["r"].debug_tiles()
    H.assert_images_close(g, o, done=o["done"], max_ambiguous=0.01, gpu_lists=(rng.numpy(), sid.numpy(), 0, 0))


def test_backward_properties_at_full_size(c2):
    gsr, r, g, cams_d, cam = c2["gsr"], c2["r"], c2["g"], c2["cams_d"], c2["cam"]
    P = cam.width * cam.height
    cfg = gsr.Config()
    gr, gd, gT = H.flat_upstream([(cam.width, cam.height)], seed=2)
    g1 = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT)))
    # translation gauge: dL/drho = R sum_i dL/dmu_i
    R = np.asarray(cam.R, np.float64)
    lhs, rhs = g1["pose"][0, :3], R @ g1["mean"].astype(np.float64).sum(0)
    assert H.rel_err(lhs, rhs) <= 1e-3, (lhs, rhs)
    # linearity in the upstream gradient
    gr2, gd2, gT2 = H.flat_upstream([(cam.width, cam.height)], seed=3)
    g2 = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(gr2), H.to_dev(gd2), H.to_dev(gT2)))
    g12 = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(gr + gr2), H.to_dev(gd + gd2),
                                              H.to_dev(gT + gT2)))
    for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        H.assert_close_scaled(g12[k], g1[k] + g2[k], what=k)
    # colour gradients sum to the accumulated opacity
    ones = np.zeros(3 * P, np.float32)
    ones[:P] = 1.0
    gc = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(ones), H.to_dev(np.zeros(P, np.float32)), None))
    A = 1.0 - c2["out"]["T_final"].double().sum().item() / P
    assert abs(gc["rgb"][:, 0].astype(np.float64).sum() / P - A) <= 1e-4 * A


def test_graph_fused_step_equals_unfused_path(c2):
    """The benchmark's launch configuration (captured fused step) gives the
    same loss and gradients as forward + L1 + backward called separately."""
    gsr, r, g, cams_d, cam = c2["gsr"], c2["r"], c2["g"], c2["cams_d"], c2["cam"]
    sizes = [(cam.width, cam.height)]
    out = c2["out"]
    t_rgb, t_d = W.noisy_targets(out["rgb"].cpu().numpy(), out["depth"].cpu().numpy(), seed=1, sigma=0.05,
                                 min_alpha=0.5, alpha=1.0 - out["T_final"].cpu().numpy())
    t_rgb, t_d = H.to_dev(t_rgb), H.to_dev(t_d)
    cfg = gsr.Config()
    # unfused reference
    r.render_forward(g, cams_d, cfg, out=out)
    loss_u, gC, gD = r.l1_loss_grad(out["rgb"], out["depth"], t_rgb, t_d, None, 1.0, 0.1)
    ref = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, gC, gD, None))
    # captured fused step, replayed twice
    grads = r.new_grads(g.n)
    loss = torch.zeros(1, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss, stream=s)
    s.synchronize()
    for rep in range(2):
        for t in grads.values():
            t.zero_()
        loss.zero_()
        torch.cuda.synchronize()
        r.graph_launch(stream=s)
        s.synchronize()
        got = H.gpu_grads_numpy(grads)
        assert abs(loss.item() - loss_u.item()) <= 1e-5 * loss_u.item()
        for k in ref:
            H.assert_close_scaled(got[k], ref[k], what=(rep, k))
    r.check_overflow(stream=s)


def test_sampled_gaussian_gradients_match_oracle(c2):
    """Exact FP64 gradients of every Gaussian, with the upstream gradient
    restricted to sampled tiles: the backward is linear in the per-pixel
    upstream values, so with zeros elsewhere the oracle backward over those
    tiles alone gives the whole gradient, also of Gaussians that cover many
    tiles (the near, large ones that carry the visible image)."""
    gsr, r, g, cams_d, cam, proj = c2["gsr"], c2["r"], c2["g"], c2["cams_d"], c2["cam"], c2["proj"]
    TX, TY = proj["TX"], proj["TY"]
    rng = np.random.default_rng(5)
    tiles = sorted(set(rng.choice(TX * TY, 20, replace=False).tolist()) | {0, TX * TY - 1})
    H_, W_ = cam.height, cam.width
    outside = np.ones((H_, W_), bool)
    for t in tiles:
        ty, tx = divmod(t, TX)
        outside[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = False
    cfg = gsr.Config()
    ocfg = O.Config().as_f32()
    fwd = O.render(c2["scene"], cam, ocfg, tiles=tiles, proj=proj, lists=c2["lists"])
    gr, gd, gT = H.flat_upstream([(W_, H_)], seed=7, zero_masks=[outside | fwd["ambiguous_grad"]])
    r.render_forward(g, cams_d, cfg)
    got = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT)))
    g2, _ = O.backward_2d(c2["scene"], cam, ocfg, gr.reshape(3, H_, W_), gd.reshape(H_, W_), gT.reshape(H_, W_),
                          fwd=fwd, tiles=tiles)
    ref = O.backward_params(proj, g2, ocfg)
    sel = np.nonzero(np.abs(g2).sum(1) > 0)[0]
    print(f"Gaussians with a gradient: {sel.size} over {len(tiles)} tiles", flush=True)
    assert sel.size >= 100, sel.size
    # nothing outside the sampled tiles may leak into the gradients
    rest = np.setdiff1d(np.arange(proj["n"]), sel)
    for k in ("mean", "rgb", "opacity_logit"):
        assert not np.any(got[k][rest]), k
    H.assert_grads_close({k: got[k][sel] for k in got if k != "pose"}, {k: ref[k][sel] for k in ref if k != "pose"})
    assert H.rel_err(got["pose"][0], ref["pose"]) <= 1e-3, (got["pose"], ref["pose"])


def test_unpacked_pair_words_four_views(gsr_lib):
    """Four views of the 300k scene (two 1920x1080, two 1200x680): 22 771
    tile keys (15 bits) and 1.2M records (21 bits) do not fit one 32-bit
    word, so the pairs are sorted as separate key and value arrays, and the
    record scan runs with its separate block-scan kernel (586 scan blocks);
    the pair count of every view equals the oracle's and its sampled tile
    lists are in-order subsequences of the oracle's keeping every Gaussian
    that reaches alpha_min in the tile."""
    gsr = gsr_lib
    scene = W.room_scene(300_000, seed=0)
    base = W.camera_replica()
    big = base.with_size(960.0, 960.0, 959.5, 539.5, 1920, 1080)
    cams = [big, W.perturb_pose(big, [0.0, 0.05, 0.15, 0.01, -0.04, 0.02]),
            W.perturb_pose(base, [-0.1, 0.02, 0.05, -0.02, 0.03, 0.01]),
            W.perturb_pose(base, [0.08, -0.03, -0.05, 0.01, 0.02, -0.03])]
    print("CASE unpacked 300k 2x1920x1080 + 2x1200x680", flush=True)
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    n_rec = len(cams) * scene.n
    assert int(tiles + 1).bit_length() + int(n_rec - 1).bit_length() > 32
    assert (n_rec + 2047) // 2048 > 512
    r = gsr.Renderer()
    r.plan(scene.n, [(c.width, c.height) for c in cams])
    r.render_forward(H.gpu_scene(gsr, scene), gsr.pack_cameras(cams), gsr.Config())
    torch.cuda.synchronize()
    rng, sid = r.debug_tiles()
    rng, sid = rng.numpy(), sid.numpy()
    total, off = 0, 0
    for v, cam in enumerate(cams):
        proj = O.project(scene, cam, O.Config().as_f32())
        assert not proj["bin_ambiguous"].any()
        lists = O.tile_lists(proj)
        total += H.rect_pairs(proj)
        T = proj["TX"] * proj["TY"]
        # every list no longer than the oracle's; sampled lists in full
        assert np.all(rng[off:off + T, 1] - rng[off:off + T, 0] <= np.diff(lists[0]))
        tiles = np.random.default_rng(v).choice(T, 24, replace=False)
        H.check_view_lists(rng, sid, off, v * scene.n, proj, lists, cam.width, cam.height, O.Config(), tiles=tiles)
        off += T
    assert r.pair_count() == total
