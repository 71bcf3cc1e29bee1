"""GPU parity of degree-1 spherical-harmonic colour (Sec. 3.1: 12
coefficients per Gaussian) against the CPU FP64 oracle, through the C ABI:
images within 1e-4, gradients of every parameter (the coefficients, and the
means and poses through the viewing direction) within 1e-3, central
differences in the smooth mode, the fused training step, pose-only mode,
and the 300k / 1200x680 workload with the upstream gradient on sampled
tiles."""
import dataclasses

import numpy as np
import pytest
import torch

import gpu_helpers as H
import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _case(gsr, sc, cams, cfg, seed=1):
    sizes = [(c.width, c.height) for c in cams]
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    out = r.render_forward(g, cams_d, cfg)
    ocfg = H.oracle_cfg_of(cfg)
    fwds = [O.render(sc, c, ocfg) for c in cams]
    rng, sid = r.debug_tiles()
    rng, sid = rng.numpy(), sid.numpy()
    tile_off = id_off = 0
    for v, (c, f) in enumerate(zip(cams, fwds)):
        H.assert_images_close(H.split_images(out, sizes)[v], f, gpu_lists=(rng, sid, tile_off, id_off))
        tile_off += f["proj"]["TX"] * f["proj"]["TY"]
        id_off += sc.n
    gr, gd, gT = H.flat_upstream(sizes, seed=seed, zero_masks=[f["ambiguous_grad"] for f in fwds])
    grads = r.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT))
    torch.cuda.synchronize()
    ref, poses = None, []
    for v, (c, f) in enumerate(zip(cams, fwds)):
        ur, ud, uT = H.view_slices(gr, gd, gT, sizes)[v]
        b = O.render_backward(sc, c, ocfg, ur, ud, uT, fwd=f)
        poses.append(b["pose"])
        ref = {k: b[k] for k in NAMES} if ref is None else {k: ref[k] + b[k] for k in NAMES}
    ref["pose"] = np.stack(poses)
    return H.gpu_grads_numpy(grads), ref, grads


def test_sh_render_and_backward_match_oracle_two_posed_views(gsr_lib):
    gsr = gsr_lib
    print("CASE sh two views", flush=True)
    sc = W.with_sh(W.random_scene(2000, seed=5, xy=1.2), seed=1)
    cams = [W.perturb_pose(W.camera_small(), [0.1, -0.05, 0.08, 0.06, 0.1, -0.05]),
            W.perturb_pose(W.camera_small().with_size(90.0, 90.0, 48.0, 31.0, 97, 63), [-0.2, 0.1, 0.0, -0.1, 0.15, 0.05])]
    got, ref, grads = _case(gsr, sc, cams, gsr.Config(bg=(0.1, 0.2, 0.3)))
    assert "rgb" not in got and np.abs(ref["sh"]).max() > 0
    H.assert_grads_close(got, ref, names=NAMES)
    for v in range(2):
        assert H.rel_err(got["pose"][v], ref["pose"][v]) <= 1e-3, (v, got["pose"][v], ref["pose"][v])


def test_sh_pose_only_mode_room_scene(gsr_lib):
    """Pose-only backward on the room scene from inside: the colour
    gradients are kept for the viewing-direction term and the pose gradient
    equals the full backward's."""
    gsr = gsr_lib
    print("CASE sh pose-only", flush=True)
    sc = W.with_sh(W.room_scene(8000, seed=4), seed=2)
    cam = W.perturb_pose(W.camera_tum_coarse(), [0.02, -0.01, 0.03, 0.01, 0.02, -0.015])
    got, ref, _ = _case(gsr, sc, [cam], gsr.Config())
    H.assert_grads_close(got, ref, names=NAMES)
    assert H.rel_err(got["pose"][0], ref["pose"][0]) <= 1e-3
    got2, _, _ = _case(gsr, sc, [cam], gsr.Config(flags=gsr.GSR_POSE_GRAD))
    assert H.rel_err(got2["pose"][0], ref["pose"][0]) <= 1e-3
    assert not np.any(got2["mean"]) and not np.any(got2["sh"])


def test_sh_backward_matches_finite_differences(gsr_lib):
    """Smooth mode: the GPU gradients of coefficients, means and the se(3)
    pose equal FP64 central differences of the oracle's forward."""
    gsr = gsr_lib
    rng = np.random.default_rng(23)
    n = 6
    T = W.se3_exp([0.2, -0.1, 0.3, 0.15, -0.2, 0.1])
    R, t = T[:3, :3].astype(np.float32), T[:3, 3].astype(np.float32)
    local = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), np.linspace(1.6, 3.4, n)], 1)
    mean = (local - t) @ R  # in front of the posed camera
    sh = np.concatenate([rng.uniform(0.5, 1.5, (n, 1, 3)), rng.normal(0, 0.5, (n, 3, 3))], axis=1)
    sc = W.Scene(mean.astype(np.float32), (np.log(0.18) + rng.normal(0, 0.3, (n, 3))).astype(np.float32),
                 rng.normal(size=(n, 4)).astype(np.float32), rng.uniform(-1.0, 1.5, n).astype(np.float32),
                 np.zeros((n, 3), np.float32), sh=sh.astype(np.float32))
    sc64 = W.Scene(*(a.astype(np.float64) for a in sc.arrays()), sh=sc.sh.astype(np.float64))
    cam = W.Camera(22.0, 22.0, 11.5, 9.5, R, t, 24, 20)
    cfg = gsr.Config.smooth(bg=(0.3, 0.6, 0.9))
    ocfg = H.oracle_cfg_of(cfg)
    r = gsr.Renderer()
    r.plan(n, [(24, 20)])
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras([cam])
    r.render_forward(g, cams_d, cfg)
    wr = np.random.default_rng(3)
    WC, WD, WT = wr.normal(size=(3, 20, 24)), wr.normal(size=(20, 24)), wr.normal(size=(20, 24))
    grads = H.gpu_grads_numpy(r.render_backward(g, cams_d, cfg, H.to_dev(WC.reshape(-1)), H.to_dev(WD.reshape(-1)),
                                                H.to_dev(WT.reshape(-1))))

    def L(s, c):
        o = O.render(s, c, ocfg)
        return float(np.sum(WC * o["rgb"]) + np.sum(WD * o["depth"]) + np.sum(WT * o["T_final"]))

    h = 1e-6
    for name in ("sh", "mean"):
        arr = getattr(sc64, name)
        flat = arr.reshape(arr.shape[0], -1)
        fd = np.zeros_like(flat)
        for i in range(flat.shape[0]):
            for j in range(flat.shape[1]):
                o0 = flat[i, j]
                flat[i, j] = o0 + h
                lp = L(sc64, cam)
                flat[i, j] = o0 - h
                lm = L(sc64, cam)
                flat[i, j] = o0
                fd[i, j] = (lp - lm) / (2 * h)
        assert H.rel_err(grads[name].reshape(fd.shape), fd) <= 1e-3, (name, H.rel_err(grads[name].reshape(fd.shape), fd))
    base = np.eye(4)
    base[:3, :3], base[:3, 3] = R.astype(np.float64), t.astype(np.float64)
    pose = np.zeros(6)
    for k in range(6):
        vals = []
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[k] = sgn * h
            Tk = W.se3_exp(xi) @ base
            vals.append(L(sc64, dataclasses.replace(cam, R=Tk[:3, :3], t=Tk[:3, 3])))
        pose[k] = (vals[0] - vals[1]) / (2 * h)
    assert H.rel_err(grads["pose"][0], pose) <= 1e-3, (grads["pose"][0], pose)


def test_sh_fused_step_matches_oracle(gsr_lib):
    """The fused forward + L1 + backward with SH colour: loss and gradients
    against the oracle's render, L1 and backward (ambiguous pixels and
    pixels whose colour error is within 1e-5 of zero masked out)."""
    gsr = gsr_lib
    print("CASE sh fused", flush=True)
    sc = W.with_sh(W.random_scene(3000, seed=6), seed=3)
    cam = W.perturb_pose(W.camera_small(), [0.05, 0.02, -0.03, 0.04, -0.02, 0.03])
    sizes = [(cam.width, cam.height)]
    ocfg = O.Config()
    f = O.render(sc, cam, ocfg)
    t_rgb, t_d, mask = W.random_targets(sizes, seed=9)
    P = cam.width * cam.height
    near = (np.abs(f["rgb"] - t_rgb.reshape(3, cam.height, cam.width)) < 1e-5).any(0) | \
        (np.abs(f["depth"] - t_d.reshape(cam.height, cam.width)) < 1e-5)
    mask = (mask.reshape(cam.height, cam.width) & ~(f["ambiguous_grad"] | near)).astype(np.uint8).reshape(-1)
    loss_o, gC, gD = O.l1_loss(f["rgb"], f["depth"], t_rgb.reshape(3, cam.height, cam.width),
                               t_d.reshape(cam.height, cam.width), mask.reshape(cam.height, cam.width))
    b = O.render_backward(sc, cam, ocfg, gC, gD, None, fwd=f)
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    loss, grads = r.render_l1_fused(H.gpu_scene(gsr, sc), gsr.pack_cameras([cam]), gsr.Config(), H.to_dev(t_rgb),
                                    H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    r.check_overflow()
    assert abs(loss.item() - loss_o) <= 1e-4 * loss_o, (loss.item(), loss_o)
    got = H.gpu_grads_numpy(grads)
    H.assert_grads_close(got, b, names=NAMES)
    assert H.rel_err(got["pose"][0], b["pose"]) <= 1e-3
    assert P > 0


def test_sh_sampled_gradients_at_full_size(gsr_lib):
    """300k Gaussians with SH colour at 1200x680: exact FP64 gradients of
    every Gaussian with the upstream gradient restricted to 20 sampled tiles
    (the backward is linear in it), and the pose."""
    gsr = gsr_lib
    print("CASE sh full size", flush=True)
    sc = W.with_sh(W.room_scene(300_000, seed=0), seed=4)
    cam = W.camera_replica()
    proj = O.project(sc, cam, O.Config().as_f32())
    lists = O.tile_lists(proj)
    TX, TY = proj["TX"], proj["TY"]
    rng = np.random.default_rng(8)
    tiles = sorted(set(rng.choice(TX * TY, 20, replace=False).tolist()) | {0, TX * TY - 1})
    H_, W_ = cam.height, cam.width
    outside = np.ones((H_, W_), bool)
    for tl in tiles:
        ty, tx = divmod(tl, TX)
        outside[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = False
    ocfg = O.Config().as_f32()
    fwd = O.render(sc, cam, ocfg, tiles=tiles, proj=proj, lists=lists)
    gr, gd, gT = H.flat_upstream([(W_, H_)], seed=7, zero_masks=[outside | fwd["ambiguous_grad"]])
    r = gsr.Renderer()
    r.plan(sc.n, [(W_, H_)])
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras([cam])
    out = r.render_forward(g, cams_d, gsr.Config())
    rg, sid = r.debug_tiles()
    H.assert_images_close(H.split_images(out, [(W_, H_)])[0], fwd, done=fwd["done"], max_ambiguous=0.01,
                          gpu_lists=(rg.numpy(), sid.numpy(), 0, 0))
    got = H.gpu_grads_numpy(r.render_backward(g, cams_d, gsr.Config(), H.to_dev(gr), H.to_dev(gd), H.to_dev(gT)))
    g2, _ = O.backward_2d(sc, cam, ocfg, gr.reshape(3, H_, W_), gd.reshape(H_, W_), gT.reshape(H_, W_), fwd=fwd,
                          tiles=tiles)
    ref = O.backward_params(proj, g2, ocfg)
    sel = np.nonzero(np.abs(g2).sum(1) > 0)[0]
    assert sel.size >= 100, sel.size
    H.assert_grads_close({k: got[k][sel] for k in NAMES}, {k: ref[k][sel] for k in NAMES}, names=NAMES)
    assert H.rel_err(got["pose"][0], ref["pose"]) <= 1e-3, (got["pose"], ref["pose"])
