"""GPU parity of the map expansion (Sec. 3.2: adding step Eq. 8, deleting
step Eq. 9) against the CPU FP64 oracle, through the C ABI.

Decisions (the unreliable-pixel mask, the order of the new Gaussians, the
decayed-Gaussian mask) must be bit-exact: both sides take them in FP64 on the
same float32 inputs.  New positions and scales are FP64 values rounded to
float32 by the kernel (checked to 1e-6 relative), colours, rotations and
initial opacities are copied (exact)."""
import numpy as np
import pytest
import torch

import gpu_helpers as H
import oracle as O
import oracle.expand as E
import workloads as W

pytestmark = pytest.mark.gpu

SENT = -12345.0


def _posed(cam, seed, scale=(0.3, 0.2)):
    rng = np.random.default_rng(seed)
    xi = np.concatenate([rng.normal(0, scale[0], 3), rng.normal(0, scale[1], 3)])
    return W.perturb_pose(cam, xi)


def _out_arrays(capacity):
    z = lambda *s: torch.full(s, SENT, device="cuda")  # noqa: E731
    return dict(mean=z(capacity, 3), log_scale=z(capacity, 3), quat=z(capacity, 4), opacity_logit=z(capacity),
                rgb=z(capacity, 3))


def _split(flat, sizes, ch=1):
    res, po = [], 0
    for w, h in sizes:
        n = w * h
        x = flat[ch * po:ch * (po + n)]
        res.append(x.reshape(ch, h, w) if ch > 1 else x.reshape(h, w))
        po += n
    return res


def _check_new(out, n, new, count):
    """Rows [n, n + count) equal the oracle's new Gaussians; others untouched."""
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    cap = got["mean"].shape[0]
    k_end = min(cap, n + count)
    sl = slice(n, k_end)
    m = k_end - n
    X = new["mean"][:m]
    np.testing.assert_allclose(got["mean"][sl], X, rtol=0, atol=1e-6 * (1.0 + np.abs(X).max()))
    np.testing.assert_allclose(got["log_scale"][sl], new["log_scale"][:m], rtol=0, atol=1e-6)
    np.testing.assert_array_equal(got["rgb"][sl], new["rgb"][:m])
    np.testing.assert_array_equal(got["quat"][sl], new["quat"][:m])
    np.testing.assert_array_equal(got["opacity_logit"][sl], np.float32(new["opacity_logit"][:m]))
    for k, v in got.items():
        assert (v[:n] == SENT).all() and (v[k_end:] == SENT).all(), k


def test_expand_add_matches_oracle_synthetic(gsr_lib):
    """Three ragged posed views (one chunk boundary inside a view, a view
    smaller than a wavefront), thresholds planted exactly in the inputs, zero
    and NaN readings: mask, count and every new Gaussian."""
    gsr = gsr_lib
    sizes = [(160, 120), (97, 53), (7, 5)]
    cams = [_posed(W.camera_small().with_size(150.0, 150.0, 79.5, 59.5, 160, 120), 1),
            _posed(W.camera_small().with_size(90.0, 80.0, 48.0, 26.0, 97, 53), 2),
            _posed(W.camera_small().with_size(6.0, 6.0, 3.0, 2.0, 7, 5), 3)]
    tau_T, tau_D, sf, li = 0.5, 0.25, 1.3, -2.0
    T, dr, do, rgb = W.expansion_images(sizes, seed=11, plant_tau_T=tau_T, plant_tau_D=tau_D)
    r = gsr.Renderer(0)
    r.plan(10, sizes)
    masks, new = E.add_gaussians(cams, _split(T, sizes), _split(dr, sizes), _split(do, sizes), _split(rgb, sizes, 3),
                                 tau_T, tau_D, sf, li)
    count_o = int(new["mean"].shape[0])
    assert count_o > 1000
    n, cap = 5, count_o + 40
    out = _out_arrays(cap)
    flag = torch.full((r.total_pixels,), 7, dtype=torch.uint8, device="cuda")
    cnt = r.expand_add(gsr.pack_cameras(cams), H.to_dev(T), H.to_dev(dr), H.to_dev(do), H.to_dev(rgb), out, n, cap,
                       tau_T, tau_D, sf, li, pixel_flag=flag)
    torch.cuda.synchronize()
    assert int(cnt.item()) == count_o
    np.testing.assert_array_equal(flag.cpu().numpy(), np.concatenate([m.ravel() for m in masks]).astype(np.uint8))
    _check_new(out, n, new, count_o)


def test_expand_add_spherical_harmonic_map(gsr_lib):
    """A map with degree-1 SH colour: the new Gaussians' coefficients (sh
    only, then sh beside rgb) equal the oracle's, the constant term rounded
    once from FP64 on both sides and the linear terms zero; capacity cuts
    the list in the middle."""
    gsr = gsr_lib
    sizes = [(160, 120), (33, 17)]
    cams = [_posed(W.camera_small().with_size(150.0, 150.0, 79.5, 59.5, 160, 120), 5),
            _posed(W.camera_small().with_size(30.0, 30.0, 16.0, 8.0, 33, 17), 6)]
    T, dr, do, rgb = W.expansion_images(sizes, seed=21)
    r = gsr.Renderer(0)
    r.plan(10, sizes)
    _, new = E.add_gaussians(cams, _split(T, sizes), _split(dr, sizes), _split(do, sizes), _split(rgb, sizes, 3),
                             0.5, 0.25, 1.0, -2.0)
    count_o = int(new["mean"].shape[0])
    assert count_o > 500
    n, cap = 2, 2 + count_o - 37
    for with_rgb in (False, True):
        out = _out_arrays(cap)
        if not with_rgb:
            del out["rgb"]
        out["sh"] = torch.full((cap, 4, 3), SENT, device="cuda")
        cnt = r.expand_add(gsr.pack_cameras(cams), H.to_dev(T), H.to_dev(dr), H.to_dev(do), H.to_dev(rgb), out, n,
                           cap, 0.5, 0.25, 1.0, -2.0)
        torch.cuda.synchronize()
        assert int(cnt.item()) == count_o
        sh = out.pop("sh").cpu().numpy()
        np.testing.assert_array_equal(sh[n:], new["sh"][:cap - n].astype(np.float32))
        assert (sh[:n] == SENT).all()
        if with_rgb:
            _check_new(out, n, new, count_o)
        else:
            got = out["mean"].cpu().numpy().astype(np.float64)
            np.testing.assert_allclose(got[n:], new["mean"][:cap - n], rtol=0,
                                       atol=1e-6 * (1.0 + np.abs(new["mean"]).max()))


def test_expand_add_capacity_empty_and_count_only(gsr_lib):
    """Capacity for half the new Gaussians: the first half is written, the
    count still reports all; no unreliable pixel: nothing written; capacity
    equal to n: only the count."""
    gsr = gsr_lib
    cam = _posed(W.camera_small(), 4)
    sizes = [(cam.width, cam.height)]
    T, dr, do, rgb = W.expansion_images(sizes, seed=12)
    r = gsr.Renderer(0)
    r.plan(10, sizes)
    cams = gsr.pack_cameras([cam])
    _, new = E.add_gaussians([cam], _split(T, sizes), _split(dr, sizes), _split(do, sizes), _split(rgb, sizes, 3),
                             0.4, 0.3, 1.0, 0.0)
    count_o = int(new["mean"].shape[0])
    n, cap = 3, 3 + count_o // 2
    out = _out_arrays(cap)
    cnt = r.expand_add(cams, H.to_dev(T), H.to_dev(dr), H.to_dev(do), H.to_dev(rgb), out, n, cap, 0.4, 0.3, 1.0, 0.0)
    torch.cuda.synchronize()
    assert int(cnt.item()) == count_o
    _check_new(out, n, new, count_o)
    # all reliable: full opacity and exact depth
    z = np.zeros_like(T)
    out = _out_arrays(50)
    cnt = r.expand_add(cams, H.to_dev(z), H.to_dev(do), H.to_dev(do), H.to_dev(rgb), out, 0, 50, 0.4, 0.3, 1.0, 0.0)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    assert all((v.cpu().numpy() == SENT).all() for v in out.values())
    cnt = r.expand_add(cams, H.to_dev(T), H.to_dev(dr), H.to_dev(do), H.to_dev(rgb), {}, 7, 7, 0.4, 0.3, 1.0, 0.0)
    torch.cuda.synchronize()
    assert int(cnt.item()) == count_o


@pytest.mark.parametrize("posed", [False, True])
def test_expand_add_after_a_render(gsr_lib, posed):
    """The adding step on a GPU render against the oracle's adding step on
    the oracle's render of the same scene: the masks agree on every pixel
    whose decision is not within the images' 1e-4 tolerance of a threshold,
    and each new Gaussian is the oracle's back-projection of its pixel."""
    gsr = gsr_lib
    cam = _posed(W.camera_small(), 7, (0.05, 0.05)) if posed else W.camera_small()
    sc = W.random_scene(2000, seed=3)
    sizes = [(cam.width, cam.height)]
    r = gsr.Renderer(0)
    r.plan(sc.n, sizes)
    cams = gsr.pack_cameras([cam])
    img = r.render_forward(H.gpu_scene(gsr, sc), cams, gsr.Config())
    orc = O.render(sc, cam, O.Config())
    _, _, do, rgb = W.expansion_images(sizes, seed=13)
    do = W.random_targets(sizes, seed=14)[1]
    tau_T, tau_D = 0.6, 0.5
    cap = cam.width * cam.height
    out = _out_arrays(cap)
    flag = torch.zeros(r.total_pixels, dtype=torch.uint8, device="cuda")
    cnt = r.expand_add(cams, img["T_final"], img["depth"], H.to_dev(do), H.to_dev(rgb), out, 0, cap, tau_T, tau_D,
                       1.0, -1.0, pixel_flag=flag)
    torch.cuda.synchronize()
    m_o = E.adding_mask(orc["T_final"].astype(np.float32), orc["depth"].astype(np.float32),
                        do.reshape(cam.height, cam.width), tau_T, tau_D)
    A = 1.0 - orc["T_final"]
    err = np.abs(do.reshape(cam.height, cam.width).astype(np.float64) - orc["depth"])
    amb = orc["ambiguous"] | (np.abs(A - tau_T) <= 1e-4) | (np.abs(err - tau_D) <= 1e-4)
    m_g = flag.cpu().numpy().reshape(cam.height, cam.width).astype(bool)
    assert not (m_g != m_o)[~amb].any()
    assert m_o.sum() > 100 and amb.mean() < 0.01
    count = int(cnt.item())
    assert count == int(m_g.sum())
    ys, xs = np.nonzero(m_g)
    got = out["mean"].cpu().numpy()[:count].astype(np.float64)
    want = np.array([E.back_project(int(x), int(y), float(do.reshape(cam.height, cam.width)[y, x]), cam)
                     for x, y in zip(xs, ys)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-6 * (1.0 + np.abs(want).max()))


def test_expand_delete_matches_oracle(gsr_lib):
    """Random posed scene, a depth image with missing readings and a Gaussian
    mask: decayed Gaussians bit-exact, new logits within float32 rounding,
    the others unchanged; in place (the output aliasing the logits) too."""
    gsr = gsr_lib
    cam = _posed(W.camera_small(), 9)
    sc = W.random_scene(5000, seed=4, z=(0.5, 6.0))
    rng = np.random.default_rng(2)
    depth = rng.uniform(1.0, 7.0, size=cam.height * cam.width).astype(np.float32)
    depth[rng.random(depth.size) < 0.1] = 0.0
    mask = (rng.random(sc.n) < 0.9).astype(np.uint8)
    gamma, eta = 0.3, 0.05
    lo, dec_o = E.delete_gaussians(sc.mean, sc.opacity_logit, cam, depth, gamma, eta, mask=mask)
    assert 200 < dec_o.sum() < sc.n - 200
    r = gsr.Renderer(0)
    g = H.gpu_scene(gsr, sc, mask=mask)
    cams = gsr.pack_cameras([cam])
    for inplace in (False, True):
        logit_out = g.opacity_logit if inplace else None
        new, dec = r.expand_delete(g, cams, H.to_dev(depth), cam.width, cam.height, gamma, eta, logit_out=logit_out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dec.cpu().numpy().astype(bool), dec_o)
        got = new.cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(got[~dec_o], sc.opacity_logit[~dec_o].astype(np.float64))
        np.testing.assert_allclose(got[dec_o], lo[dec_o], rtol=2e-7, atol=0)
        if inplace:
            assert torch.equal(g.opacity_logit, new)
        g = H.gpu_scene(gsr, sc, mask=mask)


def test_expansion_at_full_size(gsr_lib):
    """The room workload (300k Gaussians, 1200x680, the benchmark's camera):
    the adding step on seeded synthetic inputs (every pixel and new
    Gaussian) and the deleting step against the room box's own depth as the
    observation (every Gaussian: the 30 % spread through the room float in
    front of the walls)."""
    gsr = gsr_lib
    sc = W.room_scene(300_000, seed=0)
    cam = W.camera_replica()
    sizes = [(cam.width, cam.height)]
    r = gsr.Renderer(0)
    r.plan(sc.n, sizes)
    cams = gsr.pack_cameras([cam])
    T, dr, do, rgb = W.expansion_images(sizes, seed=15, plant_tau_T=0.5, plant_tau_D=0.125)
    masks, new = E.add_gaussians([cam], _split(T, sizes), _split(dr, sizes), _split(do, sizes), _split(rgb, sizes, 3),
                                 0.5, 0.125, 1.0, -2.0)
    count_o = int(new["mean"].shape[0])
    out = _out_arrays(count_o)
    out["sh"] = torch.full((count_o, 4, 3), SENT, device="cuda")  # an SH map's coefficients beside the RGB
    flag = torch.zeros(r.total_pixels, dtype=torch.uint8, device="cuda")
    print(f"adding step at full size: {count_o} new Gaussians", flush=True)
    cnt = r.expand_add(cams, H.to_dev(T), H.to_dev(dr), H.to_dev(do), H.to_dev(rgb), out, 0, count_o, 0.5, 0.125,
                       1.0, -2.0, pixel_flag=flag)
    torch.cuda.synchronize()
    assert int(cnt.item()) == count_o
    np.testing.assert_array_equal(flag.cpu().numpy(), masks[0].ravel().astype(np.uint8))
    np.testing.assert_array_equal(out.pop("sh").cpu().numpy(), new["sh"].astype(np.float32))
    _check_new(out, 0, new, count_o)
    obs = W.room_depth(cam)
    lo, dec_o = E.delete_gaussians(sc.mean, sc.opacity_logit, cam, obs, 0.3, 0.01)
    new_l, dec = r.expand_delete(H.gpu_scene(gsr, sc), cams, H.to_dev(obs), cam.width, cam.height, 0.3, 0.01)
    torch.cuda.synchronize()
    print(f"deleting step at full size: {int(dec_o.sum())} decayed", flush=True)
    np.testing.assert_array_equal(dec.cpu().numpy().astype(bool), dec_o)
    np.testing.assert_allclose(new_l.cpu().numpy()[dec_o].astype(np.float64), lo[dec_o], rtol=2e-7, atol=0)
    assert 1000 < dec_o.sum() < sc.n // 2
