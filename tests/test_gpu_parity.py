"""GPU renderer vs the CPU FP64 oracle, through the C ABI.

Bars: tile lists and their order bit-exact; colour, depth and final
transmittance within 1e-4 absolute and `last` exact on pixels whose float32
threshold decisions are unambiguous; gradients within 1e-3 relative."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _print_case(**kw):
    print("CASE", kw, flush=True)


def _check_lists(renderer, scene_list, cams, cfg_o):
    """Every tile of every view: the renderer's list against the oracle's
    rectangle list (in-order subsequence keeping every Gaussian that reaches
    alpha_min in the tile)."""
    rng, sid = renderer.debug_tiles()
    rng = rng.numpy()
    sid = sid.numpy()
    # The lists tile the sorted pairs without gaps, from position 0.
    assert rng[0, 0] == 0 and np.array_equal(rng[1:, 0], rng[:-1, 1])
    tile_off = 0
    n = renderer.n
    for v, (sc, cam) in enumerate(zip(scene_list, cams)):
        proj = O.project(sc, cam, cfg_o.as_f32())
        assert not proj["bin_ambiguous"].any()
        lists = O.tile_lists(proj)
        n_or, n_gpu, n_amb = H.check_view_lists(rng, sid, tile_off, v * n, proj, lists, cam.width, cam.height, cfg_o)
        print(f"view {v}: oracle pairs {n_or}, listed {n_gpu}, ambiguous drops {n_amb}", flush=True)
        tile_off += proj["TX"] * proj["TY"]
    return rng, sid


def _lists_of(renderer):
    rng, sid = renderer.debug_tiles()
    return rng.numpy(), sid.numpy(), 0, 0


def _max_rows_per_staged_group(proj, chunk=2048, group=128):
    """The most alpha-support rows any group of records the pair emission
    stages together holds (records in depth order; a chunk covers `chunk`
    consecutive pairs and stages its records `group` at a time; every row of
    every record needs the row test in the default mode)."""
    idx = np.nonzero(proj["valid"])[0]
    order = idx[np.lexsort((idx, proj["zbits"][idx]))]
    r = proj["rect"][order]
    cnt = (r[:, 1] - r[:, 0] + 1) * (r[:, 3] - r[:, 2] + 1)
    rows = r[:, 3] - r[:, 2] + 1
    off = np.concatenate([[0], np.cumsum(cnt)])
    best = 0
    for p0 in range(0, int(off[-1]), chunk):
        p1 = min(p0 + chunk, int(off[-1]))
        r_first = int(np.searchsorted(off, p0, side="right")) - 1
        r_last = int(np.searchsorted(off, p1 - 1, side="right")) - 1
        for rb in range(r_first, r_last + 1, group):
            best = max(best, int(rows[rb:min(rb + group, r_last + 1)].sum()))
    return best


@pytest.mark.parametrize("case", ["small", "ragged77x45", "ragged200x33", "opaque", "needles"])
def test_forward_and_lists_match_oracle(gsr_lib, case):
    gsr = gsr_lib
    if case == "small":
        sc, cam = W.random_scene(2000, seed=0), W.camera_small()
    elif case == "ragged77x45":
        sc = W.random_scene(1500, seed=3)
        cam = W.camera_small().with_size(70.0, 70.0, 38.0, 22.0, 77, 45)
    elif case == "ragged200x33":
        sc = W.random_scene(2500, seed=4, xy=1.5)
        cam = W.perturb_pose(W.camera_small().with_size(120.0, 110.0, 99.5, 16.0, 200, 33),
                             [0.05, 0.02, -0.1, 0.03, -0.05, 0.02])
    elif case == "opaque":
        sc = W.random_scene(3000, seed=5, xy=0.8, log_scale_mu=-2.5)
        sc.opacity_logit += 2.0
        cam = W.camera_small()
    else:
        # Tall thin Gaussians: the records the emission stages together hold
        # more alpha-support rows than it caches, so the rest take the
        # per-pair row test.
        sc, cam = W.needle_scene(600, seed=0), W.camera_tum()
        assert _max_rows_per_staged_group(O.project(sc, cam, O.Config().as_f32())) > 1024
    _print_case(test="forward", case=case, n=sc.n, size=(cam.width, cam.height))
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)])
    cfg = gsr.Config(bg=(0.1, 0.3, 0.2))
    out = r.render_forward(H.gpu_scene(gsr, sc), gsr.pack_cameras([cam]), cfg)
    torch.cuda.synchronize()
    g = H.split_images(out, r.sizes)[0]
    o = O.render(sc, cam, H.oracle_cfg_of(cfg))
    assert r.pair_count() == H.rect_pairs(o["proj"])
    rng, sid = _check_lists(r, [sc], [cam], H.oracle_cfg_of(cfg))
    H.assert_images_close(g, o, gpu_lists=(rng, sid, 0, 0))
    # Work totals (the roofline's FLOP count) against the oracle's walk of
    # the renderer's lists.
    work = r.work_counts(H.gpu_scene(gsr, sc), cfg)
    T = o["proj"]["TX"] * o["proj"]["TY"]
    ow = H.oracle_work(o, cam, H.oracle_cfg_of(cfg), H.gpu_view_lists(rng, sid, 0, T, 0))
    assert work["pairs"] == H.rect_pairs(o["proj"])
    assert work["bwd_evals"] == int(g["last"].sum())
    for k in ("fwd_evals", "blended"):
        assert abs(work[k] - ow[k]) <= ow["slack"], (k, work[k], ow[k], ow["slack"])
    assert ow["fwd_evals"] > 0 and ow["blended"] > 0


def test_edge_cases(gsr_lib):
    gsr = gsr_lib
    cam = W.camera_small()
    cfg = gsr.Config(bg=(0.25, 0.5, 0.75))
    # Every Gaussian culled (behind the camera): background everywhere.
    sc = W.random_scene(300, seed=1, z=(-5.0, -1.0))
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)])
    out = r.render_forward(H.gpu_scene(gsr, sc), gsr.pack_cameras([cam]), cfg)
    g = H.split_images(out, r.sizes)[0]
    assert r.pair_count() == 0
    assert np.all(g["T_final"] == 1.0) and np.all(g["depth"] == 0.0) and np.all(g["last"] == 0)
    np.testing.assert_array_equal(g["rgb"], np.broadcast_to(np.array(cfg.bg, np.float32)[:, None, None], g["rgb"].shape))
    # Non-finite parameters and zero quaternions are culled, not propagated.
    sc = W.random_scene(400, seed=2)
    sc.mean[0, 0] = np.nan
    sc.log_scale[1, 2] = np.inf
    sc.quat[2] = 0.0
    r.plan(sc.n, [(cam.width, cam.height)])
    out = r.render_forward(H.gpu_scene(gsr, sc), gsr.pack_cameras([cam]), cfg)
    g = H.split_images(out, r.sizes)[0]
    assert np.isfinite(g["rgb"]).all() and np.isfinite(g["depth"]).all()
    o = O.render(sc, cam, H.oracle_cfg_of(cfg))
    H.assert_images_close(g, o, gpu_lists=_lists_of(r))
    # A 1x1 image, a tile-aligned image, and an empty scene.
    for size in [(1, 1), (32, 32), (16, 48)]:
        sc = W.random_scene(200, seed=7)
        c2 = cam.with_size(40.0, 40.0, (size[0] - 1) / 2, (size[1] - 1) / 2, *size)
        r2 = gsr.Renderer()
        r2.plan(sc.n, [size])
        g = H.split_images(r2.render_forward(H.gpu_scene(gsr, sc), gsr.pack_cameras([c2]), cfg), r2.sizes)[0]
        H.assert_images_close(g, O.render(sc, c2, H.oracle_cfg_of(cfg)), gpu_lists=_lists_of(r2))
    r3 = gsr.Renderer()
    r3.plan(0, [(cam.width, cam.height)])
    empty = W.random_scene(0, seed=0)
    g = H.split_images(r3.render_forward(H.gpu_scene(gsr, empty), gsr.pack_cameras([cam]), cfg), r3.sizes)[0]
    assert np.all(g["T_final"] == 1.0)
    # The fused step on the empty scene, longest-first order: there is no
    # projection launch, so the work order comes from its own kernel (index
    # order first, then by the durations the first call recorded).  Every
    # pixel is background (0): the loss is the targets' own L1 over the mask.
    r3.set_tuning(4, 1, 1, 192)
    t_rgb, t_d, mask = W.random_targets(r3.sizes, seed=11)
    P = cam.width * cam.height
    m = mask.astype(bool)
    want = float(np.abs(t_rgb.astype(np.float64)).reshape(3, P)[:, m].sum()
                 + 0.1 * np.abs(t_d.astype(np.float64))[m & (t_d > 0)].sum())
    grads = r3.new_grads(0)
    for call, flags in enumerate((gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD,
                                  gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)):
        out = r3.new_images()
        grads["d_pose"].fill_(7.0 * call)  # the overwriting call must clear it
        loss, grads = r3.render_l1_fused(H.gpu_scene(gsr, empty), gsr.pack_cameras([cam]), gsr.Config(flags=flags),
                                         H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8), out=out,
                                         grads=grads)
        assert abs(loss.item() - want) <= 1e-5 * want, (call, loss.item(), want)
        assert np.all(out["T_final"].cpu().numpy() == 1.0) and np.all(out["rgb"].cpu().numpy() == 0.0), call
        assert np.all(grads["d_pose"].cpu().numpy() == 0.0), call


def test_single_gaussian_closed_form_on_gpu(gsr_lib):
    gsr = gsr_lib
    cam = dataclasses.replace(W.camera_small(), cx=70.3, cy=52.7)
    s, z, op = 0.05, 2.0, 0.8
    sc = W.Scene(np.array([[0.0, 0.0, z]], np.float32), np.full((1, 3), math.log(s), np.float32),
                 np.array([[0.6, 0.0, 0.8, 0.0]], np.float32), np.array([op], np.float32),
                 np.array([[0.9, 0.2, 0.4]], np.float32))
    r = gsr.Renderer()
    r.plan(1, [(cam.width, cam.height)])
    cfg = gsr.Config()
    g = H.split_images(r.render_forward(H.gpu_scene(gsr, sc), gsr.pack_cameras([cam]), cfg), r.sizes)[0]
    o = O.Config().as_f32()
    sig2 = (cam.fx * np.float64(np.float32(s)) / z) ** 2 + o.lowpass
    py, px = np.mgrid[0:cam.height, 0:cam.width]
    q = ((cam.cx - px) ** 2 + (cam.cy - py) ** 2) / sig2
    oo = 1 / (1 + math.exp(-np.float64(np.float32(op))))
    a = np.minimum(o.alpha_max, oo * np.exp(-0.5 * q))
    tx0, tx1 = math.floor((cam.cx - 3 * math.sqrt(sig2)) / 16), math.floor((cam.cx + 3 * math.sqrt(sig2)) / 16)
    ty0, ty1 = math.floor((cam.cy - 3 * math.sqrt(sig2)) / 16), math.floor((cam.cy + 3 * math.sqrt(sig2)) / 16)
    inl = (px // 16 >= tx0) & (px // 16 <= tx1) & (py // 16 >= ty0) & (py // 16 <= ty1)
    a = np.where(inl & (a >= o.alpha_min), a, 0.0)
    assert np.abs(g["T_final"] - (1 - a)).max() <= 1e-5
    assert np.abs(g["depth"] - a * z).max() <= 1e-4
    assert np.abs(g["rgb"][0] - 0.9 * a).max() <= 1e-5


def _backward_case(gsr, sc, cams, cfg, seed=1, approx=False):
    sizes = [(c.width, c.height) for c in cams]
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    g = H.gpu_scene(gsr, sc, mask=getattr(sc, "mask", None))
    cams_d = gsr.pack_cameras(cams)
    r.render_forward(g, cams_d, cfg)
    ocfg = H.oracle_cfg_of(cfg)
    fwds = [O.render(sc, c, ocfg) for c in cams]
    gr, gd, gT = H.flat_upstream(sizes, seed=seed, zero_masks=[f["ambiguous_grad"] for f in fwds])
    grads = r.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT))
    torch.cuda.synchronize()
    ref = None
    for v, (c, f) in enumerate(zip(cams, fwds)):
        ur, ud, uT = H.view_slices(gr, gd, gT, sizes)[v]
        b = O.render_backward(sc, c, ocfg, ur, ud, uT, approx_pose=approx, fwd=f)
        b["pose"] = b["pose"][None]
        if ref is None:
            ref = {k: b[k] for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb", "pose")}
        else:
            for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
                ref[k] = ref[k] + b[k]
            ref["pose"] = np.concatenate([ref["pose"], b["pose"]])
    return H.gpu_grads_numpy(grads), ref


def test_backward_matches_oracle_small_workload(gsr_lib):
    gsr = gsr_lib
    _print_case(test="backward", case="small")
    sc, cam = W.random_scene(2000, seed=0), W.camera_small()
    got, ref = _backward_case(gsr, sc, [cam], gsr.Config(bg=(0.2, 0.1, 0.4)))
    H.assert_grads_close(got, ref)
    for v in range(ref["pose"].shape[0]):
        assert H.rel_err(got["pose"][v], ref["pose"][v]) <= 1e-3, (got["pose"][v], ref["pose"][v])


def test_backward_matches_oracle_posed_ragged_multiview(gsr_lib):
    gsr = gsr_lib
    _print_case(test="backward", case="multiview")
    sc = W.random_scene(1500, seed=9, xy=1.2)
    cams = [W.perturb_pose(W.camera_small(), [0.02, -0.03, 0.05, 0.02, 0.01, -0.03]),
            W.camera_small().with_size(60.0, 60.0, 30.5, 20.0, 61, 41),
            W.perturb_pose(W.camera_small().with_size(100.0, 100.0, 49.5, 40.0, 100, 80), [0.0, 0.05, 0.0, -0.04, 0.0, 0.01])]
    got, ref = _backward_case(gsr, sc, cams, gsr.Config())
    H.assert_grads_close(got, ref)
    for v in range(3):
        assert H.rel_err(got["pose"][v], ref["pose"][v]) <= 1e-3


@pytest.mark.parametrize("posed", [False, True])
def test_backward_matches_oracle_room_scene(gsr_lib, posed):
    """Room scene seen from inside: Gaussians just beyond the near plane cover
    most of the image (1/z^3 terms in the chain)."""
    gsr = gsr_lib
    _print_case(test="backward", case="room", posed=posed)
    sc = W.room_scene(8000, seed=4)
    cam = W.camera_tum_coarse()
    if posed:
        cam = W.perturb_pose(cam, [0.02, -0.01, 0.03, 0.01, 0.02, -0.015])
    got, ref = _backward_case(gsr, sc, [cam], gsr.Config())
    H.assert_grads_close(got, ref)
    assert H.rel_err(got["pose"][0], ref["pose"][0]) <= 1e-3, (got["pose"][0], ref["pose"][0])
    # pose-only mode gives the same pose gradient
    got2, _ = _backward_case(gsr, sc, [cam], gsr.Config(flags=gsr.GSR_POSE_GRAD))
    assert H.rel_err(got2["pose"][0], ref["pose"][0]) <= 1e-3
    assert not np.any(got2["mean"]) and not np.any(got2["rgb"])


def test_masked_gaussians_match_oracle(gsr_lib):
    """gsr_gaussians.mask (the fine tracking stage's selection, Eq. 12):
    excluded Gaussians leave the lists, the images and the gradients --
    forward, lists and backward against the oracle with the same mask."""
    gsr = gsr_lib
    _print_case(test="masked")
    sc = W.room_scene(8000, seed=7)
    cam = W.perturb_pose(W.camera_tum_coarse(), [0.01, 0.02, -0.01, 0.01, 0.0, 0.02])
    mask = (np.random.default_rng(4).random(sc.n) > 0.4).astype(np.uint8)
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)])
    g = H.gpu_scene(gsr, sc, mask=mask)
    cams_d = gsr.pack_cameras([cam])
    cfg = gsr.Config()
    out = r.render_forward(g, cams_d, cfg)
    sc.mask = mask  # the oracle culls Gaussians with mask 0
    o = O.render(sc, cam, H.oracle_cfg_of(cfg))
    assert not o["proj"]["valid"][mask == 0].any()
    rng, sid = _check_lists(r, [sc], [cam], H.oracle_cfg_of(cfg))
    assert not np.isin(sid[:int(rng[-1, 1])], np.nonzero(mask == 0)[0]).any()
    H.assert_images_close(H.split_images(out, r.sizes)[0], o, gpu_lists=(rng, sid, 0, 0))
    got, ref = _backward_case(gsr, sc, [cam], cfg)
    H.assert_grads_close(got, ref)
    assert H.rel_err(got["pose"][0], ref["pose"][0]) <= 1e-3
    for k in ("mean", "rgb", "opacity_logit"):
        assert not np.any(got[k][mask == 0]), k


def test_paper_approx_pose_gradient(gsr_lib):
    gsr = gsr_lib
    sc, cam = W.random_scene(1000, seed=11), W.perturb_pose(W.camera_small(), [0.01, 0.0, 0.02, 0.0, 0.02, 0.0])
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_PAPER_POSE_APPROX)
    got, ref = _backward_case(gsr, sc, [cam], cfg, approx=True)
    assert H.rel_err(got["pose"][0], ref["pose"][0]) <= 1e-3


def test_backward_matches_finite_differences(gsr_lib):
    """Smooth mode: the GPU gradient equals FP64 central differences of the
    oracle's forward."""
    gsr = gsr_lib
    rng = np.random.default_rng(21)
    n = 6
    mean = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), np.linspace(1.6, 3.4, n)], 1)
    sc64 = W.Scene(mean, np.log(0.18) + rng.normal(0, 0.3, (n, 3)), rng.normal(size=(n, 4)),
                   rng.uniform(-1.0, 1.5, n), rng.random((n, 3)))
    sc = W.Scene(*(a.astype(np.float32) for a in sc64.arrays()))
    sc64 = W.Scene(*(a.astype(np.float64) for a in sc.arrays()))
    T = W.se3_exp([0.02, -0.03, 0.05, 0.03, -0.02, 0.04])
    cam = W.Camera(22.0, 22.0, 11.5, 9.5, T[:3, :3].astype(np.float32), T[:3, 3].astype(np.float32), 24, 20)
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
    fd = {}
    for name in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        arr = getattr(sc64, name)
        flat = arr.reshape(arr.shape[0], -1)
        out = np.zeros_like(flat)
        for i in range(flat.shape[0]):
            for j in range(flat.shape[1]):
                o0 = flat[i, j]
                flat[i, j] = o0 + h
                lp = L(sc64, cam)
                flat[i, j] = o0 - h
                lm = L(sc64, cam)
                flat[i, j] = o0
                out[i, j] = (lp - lm) / (2 * h)
        fd[name] = out.reshape(arr.shape)
    pose = np.zeros(6)
    base = np.eye(4)
    base[:3, :3], base[:3, 3] = cam.R.astype(np.float64), cam.t.astype(np.float64)
    for k in range(6):
        vals = []
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[k] = sgn * h
            Tk = W.se3_exp(xi) @ base
            vals.append(L(sc64, dataclasses.replace(cam, R=Tk[:3, :3], t=Tk[:3, 3])))
        pose[k] = (vals[0] - vals[1]) / (2 * h)
    for name in fd:
        assert H.rel_err(grads[name], fd[name]) <= 1e-3, (name, H.rel_err(grads[name], fd[name]))
    assert H.rel_err(grads["pose"][0], pose) <= 1e-3, (grads["pose"][0], pose)


def _fused_case(gsr, sc, cams, cfg, w_rgb=1.0, w_depth=0.1, seed=4, cap_factor=None):
    sizes = [(c.width, c.height) for c in cams]
    ocfg = H.oracle_cfg_of(cfg)
    fwds = [O.render(sc, c, ocfg) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=seed)
    # Pixels whose loss sign or threshold decisions are ambiguous in float32
    # are masked out on both sides.
    po = 0
    for (w, h), f in zip(sizes, fwds):
        n = w * h
        amb = f["ambiguous_grad"].reshape(-1).copy()
        for c in range(3):
            amb |= np.abs(f["rgb"][c].reshape(-1) - t_rgb[3 * po + c * n:3 * po + (c + 1) * n]) < 1e-4
        amb |= np.abs(f["depth"].reshape(-1) - t_d[po:po + n]) < 1e-4
        mask[po:po + n][amb] = 0
        po += n
    caps = None
    if cap_factor is not None:
        # One cap per view from the oracle's own pixel losses; pixels whose
        # loss lies within float32 reach of the cap are masked on both sides.
        caps, po = [], 0
        for (w, h), f in zip(sizes, fwds):
            n = w * h
            lp = O.l1_pixel_loss(f["rgb"], f["depth"], t_rgb[3 * po:3 * po + 3 * n].reshape(3, h, w),
                                 t_d[po:po + n].reshape(h, w), mask[po:po + n].reshape(h, w), w_rgb, w_depth)
            cap = float(O.loss_cap(lp.astype(np.float32), mask[po:po + n], cap_factor))
            caps.append(cap)
            mask[po:po + n][np.abs(lp.reshape(-1) - cap) <= 1e-4 * cap] = 0
            po += n
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    imgs = r.new_images()
    imgs["loss"] = torch.empty(sum(w * h for w, h in sizes), device="cuda")
    loss, grads = r.render_l1_fused(g, cams_d, cfg, H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8),
                                    w_rgb=w_rgb, w_depth=w_depth, out=imgs,
                                    loss_cap=None if caps is None else H.to_dev(np.array(caps, np.float32)))
    r.check_overflow()
    px_loss = imgs["loss"].cpu().numpy()
    po = 0
    for v, f in enumerate(fwds):
        w, h = sizes[v]
        n = w * h
        lp = O.l1_pixel_loss(f["rgb"], f["depth"], t_rgb[3 * po:3 * po + 3 * n].reshape(3, h, w),
                             t_d[po:po + n].reshape(h, w), mask[po:po + n].reshape(h, w), w_rgb, w_depth)
        np.testing.assert_allclose(px_loss[po:po + n], lp.reshape(-1), rtol=1e-4, atol=1e-5)
        po += n
    ref_loss, ref = 0.0, None
    po = 0
    for v, (c, f) in enumerate(zip(cams, fwds)):
        w, h = sizes[v]
        n = w * h
        l, gC, gD = O.l1_loss(f["rgb"], f["depth"], t_rgb[3 * po:3 * po + 3 * n].reshape(3, h, w),
                              t_d[po:po + n].reshape(h, w), mask[po:po + n].reshape(h, w), w_rgb, w_depth,
                              loss_cap=None if caps is None else caps[v])
        ref_loss += l
        b = O.render_backward(sc, c, ocfg, gC, gD, None, fwd=f)
        b["pose"] = b["pose"][None]
        if ref is None:
            ref = {k: b[k] for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb", "pose")}
        else:
            for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
                ref[k] = ref[k] + b[k]
            ref["pose"] = np.concatenate([ref["pose"], b["pose"]])
        po += n
    return r, float(loss.item()), ref_loss, H.gpu_grads_numpy(grads), ref


def test_fused_l1_step_matches_oracle(gsr_lib):
    gsr = gsr_lib
    _print_case(test="fused")
    sc = W.random_scene(2000, seed=0)
    cams = [W.camera_small(), W.perturb_pose(W.camera_small().with_size(90.0, 90.0, 44.5, 30.0, 90, 61),
                                             [0.03, 0.0, -0.02, 0.01, -0.02, 0.0])]
    r, loss, ref_loss, got, ref = _fused_case(gsr, sc, cams, gsr.Config(bg=(0.0, 0.1, 0.2)))
    assert abs(loss - ref_loss) <= 1e-4 * abs(ref_loss), (loss, ref_loss)
    H.assert_grads_close(got, ref)
    for v in range(2):
        assert H.rel_err(got["pose"][v], ref["pose"][v]) <= 1e-3


def test_fused_step_equals_separate_calls(gsr_lib):
    """Both backwards run their per-entry sums on the bf16 matrix cores with
    each FP32 pixel value split into a high and a low half (16 significant
    bits); the fused step feeds the upstream columns as exact residual signs
    and scales at the flush, the separate backward splits the upstream
    gradients themselves.  On the room scene from the TUM camera (two views)
    the two agree far inside the oracle tolerance: gradients to 1e-4
    relative plus 5e-5 of each tensor's scale, losses and images exactly."""
    gsr = gsr_lib
    sc = W.room_scene(20_000, seed=5)
    cams = [W.camera_tum(), W.perturb_pose(W.camera_tum(), np.array([0.03, -0.02, 0.01, 0.02, 0.01, -0.03]))]
    sizes = [(c.width, c.height) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=8)
    w_rgb, w_depth = 0.9, 0.2
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    args = (H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    rf = gsr.Renderer()
    rf.plan(sc.n, sizes)
    imgs_f = rf.new_images()
    loss_f, grads_f = rf.render_l1_fused(g, cams_d, cfg, *args, w_rgb=w_rgb, w_depth=w_depth, out=imgs_f)
    rs = gsr.Renderer()
    rs.plan(sc.n, sizes)
    imgs_s = rs.render_forward(g, cams_d, cfg)
    loss_s, gC, gD = rs.l1_loss_grad(imgs_s["rgb"], imgs_s["depth"], *args, w_rgb=w_rgb, w_depth=w_depth)
    grads_s = rs.render_backward(g, cams_d, cfg, gC, gD)
    torch.cuda.synchronize()
    for k in ("rgb", "depth"):
        assert torch.equal(imgs_f[k], imgs_s[k]), k
    assert float(loss_f.item()) == pytest.approx(float(loss_s.item()), rel=1e-6)
    a, b = H.gpu_grads_numpy(grads_f), H.gpu_grads_numpy(grads_s)
    for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb", "pose"):
        assert np.abs(b[k]).max() > 0, k
        assert H.rel_err(a[k], b[k]) <= 1e-4, (k, H.rel_err(a[k], b[k]))
        H.assert_close_scaled(a[k], b[k], rtol=1e-4, scale_tol=5e-5, what=k)


def test_fused_l1_step_with_loss_cap_matches_oracle(gsr_lib):
    """Outlier rejection: with a per-view cap at 1.5x the median pixel loss
    about a quarter of the pixels leave the loss and the backward."""
    gsr = gsr_lib
    _print_case(test="fused-cap")
    sc = W.random_scene(2000, seed=0)
    cams = [W.camera_small(), W.perturb_pose(W.camera_small().with_size(90.0, 90.0, 44.5, 30.0, 90, 61),
                                             [0.03, 0.0, -0.02, 0.01, -0.02, 0.0])]
    r, loss, ref_loss, got, ref = _fused_case(gsr, sc, cams, gsr.Config(), w_rgb=0.8, w_depth=0.3,
                                              cap_factor=1.5)
    assert abs(loss - ref_loss) <= 1e-4 * abs(ref_loss), (loss, ref_loss)
    H.assert_grads_close(got, ref)
    for v in range(2):
        assert H.rel_err(got["pose"][v], ref["pose"][v]) <= 1e-3


def test_loss_median_matches_oracle(gsr_lib):
    """Exact per-view lower median (radix select) on synthetic loss images:
    ties, zeros, -0 and negatives, +inf and NaN, masks, a single pixel and a
    view without eligible pixels."""
    gsr = gsr_lib
    sizes = [(37, 23), (160, 120), (1, 1), (16, 16), (64, 48), (640, 480), (33, 17)]
    px, mask = W.loss_images(sizes, seed=3)
    r = gsr.Renderer()
    r.plan(1, sizes)
    for use_mask in (False, True):
        for factor in (10.0, 1.0):
            caps = r.loss_median(H.to_dev(px), H.to_dev(mask, torch.uint8) if use_mask else None, factor).cpu()
            po = 0
            for v, (w, h) in enumerate(sizes):
                n = w * h
                want = O.loss_cap(px[po:po + n], mask[po:po + n] if use_mask else None, factor)
                got = np.float32(caps[v].item())
                assert (np.isnan(want) and np.isnan(got)) or got == want, (v, use_mask, factor, got, want)
                po += n


def test_l1_loss_grad_exact_signs(gsr_lib):
    gsr = gsr_lib
    sizes = [(37, 21), (16, 16)]
    rng = np.random.default_rng(0)
    P = sum(w * h for w, h in sizes)
    rgb = rng.random(3 * P).astype(np.float32)
    dep = rng.uniform(0, 3, P).astype(np.float32)
    trgb, tdep, mask = W.random_targets(sizes, seed=2)
    trgb[:10] = rgb[:10]  # exact ties: sign(0) = 0
    mask[5:40] = 0
    r = gsr.Renderer()
    r.plan(10, sizes)
    loss, gC, gD = r.l1_loss_grad(H.to_dev(rgb), H.to_dev(dep), H.to_dev(trgb), H.to_dev(tdep),
                                  H.to_dev(mask, torch.uint8), 0.8, 0.3)
    po, ref_loss = 0, 0.0
    gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    for w, h in sizes:
        n = w * h
        l, c, d = O.l1_loss(rgb[3 * po:3 * po + 3 * n].reshape(3, h, w), dep[po:po + n].reshape(h, w),
                            trgb[3 * po:3 * po + 3 * n].reshape(3, h, w), tdep[po:po + n].reshape(h, w),
                            mask[po:po + n].reshape(h, w), 0.8, 0.3)
        ref_loss += l
        np.testing.assert_array_equal(gC[3 * po:3 * po + 3 * n], c.reshape(-1).astype(np.float32))
        np.testing.assert_array_equal(gD[po:po + n], d.reshape(-1).astype(np.float32))
        po += n
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss


def test_batched_views_equal_separate_calls(gsr_lib):
    gsr = gsr_lib
    sc = W.room_scene(20000, seed=0)
    cams = W.mapping_views(seed=2)[:3]
    cams = [c.with_size(c.fx / 4, c.fy / 4, (c.cx + 0.5) / 4 - 0.5, (c.cy + 0.5) / 4 - 0.5, c.width // 4, c.height // 4)
            for c in cams]
    sizes = [(c.width, c.height) for c in cams]
    cfg = gsr.Config()
    g = H.gpu_scene(gsr, sc)
    rb = gsr.Renderer()
    rb.plan(sc.n, sizes)
    cams_d = gsr.pack_cameras(cams)
    outb = H.split_images(rb.render_forward(g, cams_d, cfg), sizes)
    gr, gd, gT = H.flat_upstream(sizes, seed=3)
    gb = H.gpu_grads_numpy(rb.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT)))
    acc = None
    for v, c in enumerate(cams):
        r1 = gsr.Renderer()
        r1.plan(sc.n, [sizes[v]])
        c_d = gsr.pack_cameras([c])
        o1 = H.split_images(r1.render_forward(g, c_d, cfg), [sizes[v]])[0]
        for k in ("rgb", "depth", "T_final", "last"):
            np.testing.assert_array_equal(o1[k], outb[v][k])
        ur, ud, uT = H.view_slices(gr, gd, gT, sizes)[v]
        g1 = H.gpu_grads_numpy(r1.render_backward(g, c_d, cfg, H.to_dev(ur.reshape(-1)), H.to_dev(ud.reshape(-1)),
                                                  H.to_dev(uT.reshape(-1))))
        H.assert_close_scaled(gb["pose"][v], g1["pose"][0], what="pose")
        if acc is None:
            acc = g1
        else:
            for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
                acc[k] = acc[k] + g1[k]
    for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
        H.assert_close_scaled(gb[k], acc[k], what=k)


def test_batch_sizes_equal(gsr_lib):
    """Every staged batch size of the fused rasteriser gives the default's
    images exactly and its loss and gradients up to the order of the FP64
    additions; other sizes are refused."""
    gsr = gsr_lib
    sc = W.room_scene(20000, seed=6)
    base = W.camera_tum_coarse()
    cams = [W.perturb_pose(base, [0.015 * v, -0.01 * (v % 2), 0.02 * (v % 3), 0.003 * v, 0.0, -0.002 * v])
            for v in range(6)]
    sizes = [(c.width, c.height) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=10)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    args = (H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    for bad in (32, 100, 320):
        with pytest.raises(gsr.GsrError) as e:
            r.set_tuning(4, 1, 1, bad)
        assert e.value.status == gsr.GSR_E_INVALID
    results = {}
    for batch in (192, 64, 128, 256):
        r.set_tuning(4, 1, 1, batch)
        assert r.get_tuning()["batch"] == batch
        out = r.new_images()
        loss, grads = r.render_l1_fused(g, cams_d, cfg, *args, out=out)
        results[batch] = ({k: v.cpu().numpy() for k, v in out.items() if v is not None}, loss.item(),
                          H.gpu_grads_numpy(grads))
    img0, loss0, ref = results[192]
    for batch in (64, 128, 256):
        img, loss, got = results[batch]
        for k, v in img0.items():
            np.testing.assert_array_equal(img[k], v, err_msg=f"batch {batch} {k}")
        assert abs(loss - loss0) <= 1e-5 * abs(loss0), batch
        for k in ref:
            H.assert_close_scaled(got[k], ref[k], what=(batch, k))


def test_longest_first_order_equals_index_order(gsr_lib):
    """The persistent rasteriser's longest-first tile order (index order on a
    fresh workspace, then by the durations the previous fused step recorded)
    gives the index order's images exactly and its loss and gradients up to
    the order of the FP64 additions, over many views."""
    gsr = gsr_lib
    sc = W.room_scene(20000, seed=5)
    base = W.camera_tum_coarse()
    cams = [W.perturb_pose(base, [0.02 * (v % 3), -0.01 * (v % 2), 0.01 * v, 0.004 * v, -0.003 * (v % 4), 0.0])
            for v in range(12)]
    sizes = [(c.width, c.height) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=9)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    args = (H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    r0 = gsr.Renderer()
    r0.plan(sc.n, sizes)
    r0.set_tuning(2, 1, 0)
    out0 = r0.new_images()
    loss0, grads0 = r0.render_l1_fused(g, cams_d, cfg, *args, out=out0)
    ref = H.gpu_grads_numpy(grads0)
    img0 = {k: v.cpu().numpy() for k, v in out0.items() if v is not None}
    r1 = gsr.Renderer()  # fresh workspace: no recorded durations yet
    r1.plan(sc.n, sizes)
    r1.set_tuning(2, 1, 1)
    out1 = r1.new_images()
    grads1 = r1.new_grads(sc.n)
    loss1 = torch.zeros(1, device="cuda")
    for call in range(3):
        r1.render_l1_fused(g, cams_d, cfg, *args, out=out1, grads=grads1, loss=loss1)
        for k, v in img0.items():
            np.testing.assert_array_equal(out1[k].cpu().numpy(), v, err_msg=f"call {call} {k}")
        assert abs(loss1.item() - loss0.item()) <= 1e-5 * abs(loss0.item()), call
        got = H.gpu_grads_numpy(grads1)
        for k in ref:
            H.assert_close_scaled(got[k], ref[k], what=(call, k))


@pytest.mark.parametrize("n_views", [2, 48])
def test_overwrite_mode_equals_accumulation_into_zeros(gsr_lib, n_views):
    """GSR_GRAD_OVERWRITE: a fused step into buffers holding garbage gives the
    gradients and loss that the accumulating mode adds into zeroed buffers,
    on two calls in a row and on graph replays (2 and 48 views)."""
    gsr = gsr_lib
    sc = W.room_scene(3000, seed=4)
    base = W.camera_tum_coarse()
    base = base.with_size(base.fx / 3, base.fy / 3, 26.5, 19.5, 54, 40)
    cams = [W.perturb_pose(base, [0.01 * (v % 5), -0.004 * (v % 3), 0.002 * v, 0.003 * (v % 4), 0.0, 0.001 * v])
            for v in range(n_views)]
    sizes = [(c.width, c.height) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=8)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    args = (H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    loss_a, grads_a = r.render_l1_fused(g, cams_d, gsr.Config(), *args)
    ref = H.gpu_grads_numpy(grads_a)
    ref_loss = loss_a.item()
    assert np.abs(ref["pose"]).sum() > 0
    cfg_o = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)

    def check(grads, loss, what):
        got = H.gpu_grads_numpy(grads)
        for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb", "pose"):
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-5, atol=1e-6 * float(np.abs(ref[k]).max()),
                                       err_msg=f"{what} {k}")
        assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss), what

    grads = r.new_grads(sc.n)
    loss = torch.full((1,), 5.0, device="cuda")
    for t in grads.values():
        t.fill_(7.0)
    for call in range(2):
        r.render_l1_fused(g, cams_d, cfg_o, *args, grads=grads, loss=loss)
        check(grads, loss, f"eager call {call}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r.graph_capture(g, cams_d, cfg_o, *args, grads=grads, loss=loss, stream=s)
    s.synchronize()
    for rep in range(3):
        for t in grads.values():
            t.fill_(-3.0)
        torch.cuda.synchronize()
        r.graph_launch(stream=s)
        s.synchronize()
        check(grads, loss, f"graph replay {rep}")


def test_graph_replay_matches_eager(gsr_lib):
    gsr = gsr_lib
    sc = W.room_scene(30000, seed=1)
    cams = [W.camera_tum_coarse(), W.perturb_pose(W.camera_tum_coarse(), [0.02, 0.0, 0.0, 0.0, 0.01, 0.0])]
    sizes = [(c.width, c.height) for c in cams]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=5)
    g = H.gpu_scene(gsr, sc)
    cams_d = gsr.pack_cameras(cams)
    cfg = gsr.Config()
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    args = (H.to_dev(t_rgb), H.to_dev(t_d), H.to_dev(mask, torch.uint8))
    loss_e, grads_e = r.render_l1_fused(g, cams_d, cfg, *args)
    ref = H.gpu_grads_numpy(grads_e)
    ref_loss = loss_e.item()
    s = torch.cuda.Stream()
    grads = r.new_grads(sc.n)
    loss = torch.zeros(1, device="cuda")
    with torch.cuda.stream(s):
        r.graph_capture(g, cams_d, cfg, *args, grads=grads, loss=loss, stream=s)
    s.synchronize()
    for rep in range(3):
        for t in grads.values():
            t.zero_()
        loss.zero_()
        torch.cuda.synchronize()
        r.graph_launch(stream=s)
        s.synchronize()
        # some eager work between replays
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()
        got = H.gpu_grads_numpy(grads)
        assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss), rep
        for k in ref:
            H.assert_close_scaled(got[k], ref[k], what=(rep, k))
    r.check_overflow(stream=s)


def test_capacity_overflow_reports_required_pairs(gsr_lib):
    gsr = gsr_lib
    sc, cam = W.random_scene(2000, seed=0), W.camera_small()
    need = H.rect_pairs(O.project(sc, cam, O.Config().as_f32()))
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)], pair_capacity=1000)
    lib = r.lib
    import ctypes
    g = H.gpu_scene(gsr, sc)
    out = r.new_images()
    ws, wsb = r._ws()
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.gsr_render_forward(r.ctx, ctypes.byref(g.c()), gsr.pack_cameras([cam]).data_ptr(), 1,
                                ctypes.byref(gsr.Config().to_c()), ws, wsb, ctypes.byref(r._images_c(out)), stream)
    assert st == gsr.GSR_OK  # asynchronous: the overflow is recorded on the device
    assert lib.gsr_check_overflow(r.ctx, ws, stream) == gsr.GSR_E_CAPACITY
    assert r.required_pairs() == need
    assert lib.gsr_check_overflow(r.ctx, ws, stream) == gsr.GSR_OK  # reported once
    # The binding grows the buffer and succeeds.
    o = H.split_images(r.render_forward(g, gsr.pack_cameras([cam]), gsr.Config()), r.sizes)[0]
    H.assert_images_close(o, O.render(sc, cam), gpu_lists=_lists_of(r))


def test_invalid_arguments_and_call_order(gsr_lib):
    gsr = gsr_lib
    import ctypes
    sc, cam = W.random_scene(100, seed=0), W.camera_small()
    r = gsr.Renderer()
    r.plan(50, [(cam.width, cam.height)])  # wrong n
    g = H.gpu_scene(gsr, sc)
    with pytest.raises(gsr.GsrError) as e:
        r.render_forward(g, gsr.pack_cameras([cam]), gsr.Config())
    assert e.value.status == gsr.GSR_E_INVALID
    r.plan(100, [(cam.width, cam.height)])
    P = cam.width * cam.height
    with pytest.raises(gsr.GsrError) as e:  # backward before any forward
        r.render_backward(g, gsr.pack_cameras([cam]), gsr.Config(), torch.zeros(3 * P, device="cuda"),
                          torch.zeros(P, device="cuda"))
    assert e.value.status == gsr.GSR_E_STATE
    for bad in (dict(alpha_max=1.5), dict(alpha_min=1.5), dict(alpha_min=float("nan"))):
        with pytest.raises(gsr.GsrError) as e:
            r.render_forward(g, gsr.pack_cameras([cam]), gsr.Config(**bad))
        assert e.value.status == gsr.GSR_E_INVALID, bad
    ws, wsb = r._ws()
    assert r.lib.gsr_render_forward(r.ctx, ctypes.byref(g.c()), gsr.pack_cameras([cam]).data_ptr(), 1,
                                    ctypes.byref(gsr.Config().to_c()), ws, wsb - 4096, None, None) == gsr.GSR_E_INVALID
    # The binding rejects device buffers shorter than the plan needs (the
    # kernels cannot see a tensor's length), before anything is launched.
    P = cam.width * cam.height
    short = torch.zeros(1, device="cuda")
    with pytest.raises(ValueError):
        r.render_backward(g, gsr.pack_cameras([cam]), gsr.Config(), short, torch.zeros(P, device="cuda"))
    with pytest.raises(ValueError):
        r.l1_loss_grad(torch.zeros(3 * P, device="cuda"), short, torch.zeros(3 * P, device="cuda"),
                       torch.zeros(P, device="cuda"))
    with pytest.raises(ValueError):
        r.render_l1_fused(g, gsr.pack_cameras([cam]), gsr.Config(), torch.zeros(3 * P, device="cuda"), short)
    with pytest.raises(ValueError):
        r.render_forward(g, short, gsr.Config())


@pytest.mark.parametrize("case", ["one-view", "two-views-xi", "pose-only"])
def test_autograd_function(gsr_lib, case):
    """torch.autograd.Function boundary against the oracle at 1e-3: all
    parameter gradients and the gradient of pose_xi (cameras at
    Exp(xi) T0, the xi gradient J_l(xi)^T times the oracle's left-perturbation
    gradient at that pose), ambiguous pixels masked on both sides."""
    gsr = gsr_lib
    sc = W.random_scene(800, seed=2)
    cams0 = [W.camera_small()]
    xi = np.zeros((1, 6))
    if case == "two-views-xi":
        cams0.append(W.perturb_pose(W.camera_small().with_size(90.0, 90.0, 44.5, 30.0, 90, 61),
                                    [0.03, 0.0, -0.02, 0.01, -0.02, 0.0]))
        xi = np.array([[0.02, -0.01, 0.03, 0.02, 0.01, -0.015], [-0.01, 0.02, 0.0, 0.0, 0.03, 0.01]])
    _print_case(test="autograd", case=case)
    sizes = [(c.width, c.height) for c in cams0]
    xi = xi.astype(np.float32)
    # The poses the renderer sees: Exp(xi) T0 in FP64, rounded to float32.
    cams = []
    for c, x in zip(cams0, xi):
        R, t = O.apply_xi(x.astype(np.float64), np.asarray(c.R, np.float64), np.asarray(c.t, np.float64))
        cams.append(dataclasses.replace(c, R=R.astype(np.float32), t=t.astype(np.float32)))
    cfg = gsr.Config() if case != "pose-only" else gsr.Config(flags=gsr.GSR_POSE_GRAD)
    r = gsr.Renderer()
    r.plan(sc.n, sizes)
    params = [H.to_dev(a).requires_grad_(True) for a in sc.arrays()]
    xi_d = H.to_dev(xi).requires_grad_(True)
    rgb, depth, T = gsr.render(r, *params, gsr.pack_cameras(cams0), cfg=cfg, pose_xi=xi_d)
    fwds = [O.render(sc, c) for c in cams]
    gr, gd, gT = H.flat_upstream(sizes, seed=6, zero_masks=[f["ambiguous_grad"] for f in fwds])
    (rgb * H.to_dev(gr)).sum().add((depth * H.to_dev(gd)).sum()).add((T * H.to_dev(gT)).sum()).backward()
    ref = None
    for v, (c, f) in enumerate(zip(cams, fwds)):
        ur, ud, uT = H.view_slices(gr, gd, gT, sizes)[v]
        assert f["ambiguous_grad"].mean() < 5e-3
        b = O.render_backward(sc, c, O.Config(), ur, ud, uT, fwd=f)
        b["xi"] = O.pose_xi_grad(xi[v].astype(np.float64), b["pose"])
        if ref is None:
            ref = {k: b[k] for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb")}
            ref["xi"] = [b["xi"]]
        else:
            for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb"):
                ref[k] = ref[k] + b[k]
            ref["xi"].append(b["xi"])
    if case == "pose-only":
        for p in params:
            assert p.grad is None or not torch.any(p.grad)
    else:
        H.assert_grads_close({k: p.grad.cpu().numpy() for p, k in zip(params, ("mean", "log_scale", "quat",
                                                                                 "opacity_logit", "rgb"))}, ref)
    for v in range(len(cams)):
        assert H.rel_err(xi_d.grad.cpu().numpy()[v], ref["xi"][v]) <= 1e-3, (v, xi_d.grad[v], ref["xi"][v])


def test_backward_of_an_overwritten_forward_is_refused(gsr_lib):
    """Two autograd renders on one renderer before either backward: the
    first call's state has been overwritten, so its backward raises
    GSR_E_STATE instead of returning the second call's gradients; the second
    call's backward is unaffected."""
    gsr = gsr_lib
    sc, cam = W.random_scene(500, seed=3), W.camera_small()
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)])
    cams = gsr.pack_cameras([cam])
    p1 = [H.to_dev(a).requires_grad_(True) for a in sc.arrays()]
    p2 = [H.to_dev(a).requires_grad_(True) for a in sc.arrays()]
    out1 = gsr.render(r, *p1, cams)
    out2 = gsr.render(r, *p2, cams)
    with pytest.raises(gsr.GsrError) as e:
        out1[0].sum().backward()
    assert e.value.status == gsr.GSR_E_STATE
    out2[0].sum().backward()
    f = O.render(sc, cam)
    gC = np.zeros((3, cam.height, cam.width))
    gC[:, ~f["ambiguous_grad"]] = 1.0
    ok = H.to_dev(gC.reshape(-1))
    for p in p2:
        p.grad = None
    out3 = gsr.render(r, *p2, cams)
    (out3[0] * ok).sum().backward()
    ref = O.render_backward(sc, cam, O.Config(), gC, np.zeros((cam.height, cam.width)), None, fwd=f)
    assert H.rel_err(p2[0].grad.cpu().numpy(), ref["mean"]) <= 1e-3


def test_reliable_selection_bit_exact(gsr_lib):
    gsr = gsr_lib
    sc = W.room_scene(20000, seed=3)
    cam = W.perturb_pose(W.camera_tum(), [0.01, 0.02, -0.03, 0.01, -0.02, 0.01])
    _, depth, _ = W.random_targets([(cam.width, cam.height)], seed=4, depth_range=(0.3, 4.0))
    mask = (np.random.default_rng(0).random(sc.n) > 0.1).astype(np.uint8)
    r = gsr.Renderer()
    r.plan(sc.n, [(cam.width, cam.height)])
    g = H.gpu_scene(gsr, sc, mask=mask)
    got = r.select_reliable(g, gsr.pack_cameras([cam]), H.to_dev(depth), cam.width, cam.height, 0.1).cpu().numpy()
    ref = O.select_reliable(sc, cam, depth, 0.1, mask=mask)
    assert 0 < ref.sum() < sc.n
    np.testing.assert_array_equal(got, ref)
