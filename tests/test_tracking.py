"""Coarse-to-fine tracking driver: the device-side SE(3) exponential (CPU
check against the generator's) and, on the GPU, convergence of a perturbed
pose towards the pose the target was rendered from."""
import math

import numpy as np
import pytest
import torch

import workloads as W


def _rot_angle(R):
    return math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(R) - 1) / 2))))


def test_se3_exp_matches_reference():
    from paper_2311_11700_amd.tracking import se3_exp
    rng = np.random.default_rng(0)
    for scale in (1e-9, 1e-3, 0.3, 2.0):
        xi = rng.normal(size=6) * scale
        got = se3_exp(torch.tensor(xi, dtype=torch.float64)).numpy()
        np.testing.assert_allclose(got, W.se3_exp(xi), atol=1e-12)


def test_downsample_targets_box_average():
    from paper_2311_11700_amd.tracking import downsample_targets
    rgb = torch.arange(3 * 8 * 8, dtype=torch.float32)
    d = torch.ones(64)
    d[0] = 0.0
    d[1] = 3.0
    c, dd = downsample_targets(rgb, d, 8, 8, 4)
    assert c.shape == (3 * 4,) and dd.shape == (4,)
    block = rgb.reshape(3, 8, 8)[0, :4, :4]
    assert abs(c[0].item() - block.mean().item()) < 1e-6
    assert abs(dd[0].item() - (14 * 1.0 + 3.0) / 15) < 1e-6  # the invalid reading is skipped


@pytest.mark.gpu
def test_tracking_converges(gsr_lib):
    """The map holds flat Gaussians on the room's floor and walls plus 5%
    outliers 0.3-0.6 m off the surfaces; the observation is rendered (at the
    true pose) from the surfaces only, with 10% of the depth readings missing.
    The fine stage's Eq. 12 selection drops the outliers that disagree with
    the observed depth, and the pose converges."""
    gsr = gsr_lib
    from paper_2311_11700_amd.tracking import Tracker, TrackingConfig
    print("CASE tracking 60k room (5% outliers) 640x480", flush=True)
    n = 60_000
    scene, n_surf = W.tracking_scene(n, seed=0, outlier_fraction=0.05, offset=(0.3, 0.6))
    truth = W.camera_tracking()
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    surf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    surf[:n_surf] = 1
    r = gsr.Renderer()
    r.plan(n, [(truth.width, truth.height)])
    out = r.render_forward(gsr.Gaussians(g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb, surf),
                           gsr.pack_cameras([truth]), gsr.Config())
    t_rgb = out["rgb"].clone()
    t_d = out["depth"].clone()
    rng = np.random.default_rng(3)
    t_d[torch.as_tensor(rng.random(t_d.numel()) < 0.1, device="cuda")] = 0.0
    Tt = np.eye(4)
    Tt[:3, :3], Tt[:3, 3] = truth.R, truth.t
    # outliers whose centre lands in the image (the ones Eq. 12 can judge)
    Xc = scene.mean.astype(np.float64) @ np.asarray(truth.R, np.float64).T + np.asarray(truth.t, np.float64)
    u = truth.fx * Xc[:, 0] / Xc[:, 2] + truth.cx
    v = truth.fy * Xc[:, 1] / Xc[:, 2] + truth.cy
    seen = (Xc[:, 2] > 0.2) & (u > 0) & (u < truth.width - 1) & (v > 0) & (v < truth.height - 1)
    seen[:n_surf] = False
    for seed in (2, 5):
        start = W.tracking_start(seed=seed, truth=truth, trans=0.01, rot_deg=0.5)
        T0 = np.eye(4)
        T0[:3, :3], T0[:3, 3] = start.R, start.t
        tr = Tracker(g, truth, TrackingConfig(reliable_eps=0.3, fine_iters=195))
        losses = []
        T = tr.track(torch.tensor(T0), t_rgb, t_d, losses=losses).cpu().numpy()
        kept = tr.reliable.cpu().numpy().astype(bool)
        E0 = T0 @ np.linalg.inv(Tt)
        E1 = T @ np.linalg.inv(Tt)
        e0_t, e1_t = np.linalg.norm(E0[:3, 3]), np.linalg.norm(E1[:3, 3])
        e0_r, e1_r = _rot_angle(E0[:3, :3]), _rot_angle(E1[:3, :3])
        print(f"seed {seed}: reliable surfaces {kept[:n_surf].sum()}/{n_surf}, outliers in view "
              f"{kept[seen].sum()}/{seen.sum()}; translation {e0_t * 100:.3f} -> {e1_t * 100:.3f} cm, rotation "
              f"{e0_r:.3f} -> {e1_r:.3f} deg, loss {losses[5].item():.1f} -> {losses[-1].item():.1f}", flush=True)
        assert kept[:n_surf].mean() > 0.99 and kept[seen].mean() < 0.5
        assert e1_t < 0.5 * e0_t and e1_r < 0.5 * e0_r
        assert losses[-1].item() < losses[5].item()
