"""The allocation-free fused step (gsr_render_l1_fused_noalloc) against the
fused step with a caller workspace (gsr_render_l1_fused), through the C ABI.

Both calls run the same kernels on the same plan; only the workspace differs
(the library's static scratch against a torch allocation).  Two calls in a
row, the second on a smaller workload (fewer Gaussians, a smaller image, a
re-plan in between), so the second reads a scratch that still holds the
first call's state.  Images must agree bit for bit (the forward is
deterministic); the loss and the gradients, whose FP64 sums over tiles are
added in tile-completion order, to 1e-5 of their scale (the oracle bar for
gradients is 1e-3).
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import gpu_scene

pytestmark = pytest.mark.gpu

FLAGS_ALL = 1 << 1 | 1 << 2  # GSR_GAUSS_GRAD | GSR_POSE_GRAD


def _case(gsr, n, cam, seed):
    sc = W.random_scene(n, seed=seed)
    sizes = [(cam.width, cam.height)]
    t_rgb, t_d, mask = W.random_targets(sizes, seed=seed + 1)
    return sc, sizes, [torch.as_tensor(a).cuda() for a in (t_rgb, t_d, mask)]


def _run(r, gsr, g, cams, cfg, tg, noalloc):
    P = r.total_pixels
    out = dict(rgb=torch.full((3 * P,), -1.0, device="cuda"), depth=torch.full((P,), -1.0, device="cuda"),
               T_final=torch.full((P,), -1.0, device="cuda"),
               last=torch.full((P,), -7, dtype=torch.int32, device="cuda"),
               loss=torch.full((P,), -1.0, device="cuda"))
    grads = r.new_grads(g.n)
    loss = torch.zeros(1, device="cuda")
    if noalloc:
        r.render_l1_fused_noalloc(g, cams, cfg, *tg, out=out, grads=grads, loss=loss)
        r.check_overflow_noalloc()
    else:
        r.render_l1_fused(g, cams, cfg, *tg, out=out, grads=grads, loss=loss)
        r.check_overflow()
    torch.cuda.synchronize()
    return out, grads, loss


def _compare(a, b):
    out_a, gr_a, loss_a = a
    out_b, gr_b, loss_b = b
    for k in ("rgb", "depth", "T_final", "last", "loss"):
        np.testing.assert_array_equal(out_a[k].cpu().numpy(), out_b[k].cpu().numpy(), err_msg=k)
    la, lb = float(loss_a.item()), float(loss_b.item())
    assert abs(la - lb) <= 1e-5 * max(abs(lb), 1e-30), (la, lb)
    for k, v in gr_b.items():
        x, y = gr_a[k].cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        scale = max(np.abs(y).max(), 1e-30)
        err = np.abs(x - y).max() / scale
        assert err <= 1e-5, (k, err)
        assert np.isfinite(x).all()


def test_noalloc_matches_workspace_step_two_calls(gsr_lib):
    gsr = gsr_lib
    r = gsr.Renderer(0)
    cfg = gsr.Config(flags=FLAGS_ALL)
    cases = [(900, W.camera_small(), 0),
             (300, W.camera_small().with_size(70.0, 70.0, 47.5, 31.5, 96, 64), 5)]
    for n, cam, seed in cases:
        print(f"no-alloc fused step: n={n}, {cam.width}x{cam.height}, seed {seed}", flush=True)
        sc, sizes, tg = _case(gsr, n, cam, seed)
        need = r.plan(sc.n, sizes)
        assert need <= gsr.GSR_NOALLOC_SCRATCH_BYTES, need
        g = gpu_scene(gsr, sc)
        cams = gsr.pack_cameras([cam])
        # The static-scratch call first, so that the second case reads a
        # scratch left by the first case's (larger) plan.
        b = _run(r, gsr, g, cams, cfg, tg, noalloc=True)
        a = _run(r, gsr, g, cams, cfg, tg, noalloc=False)
        _compare(b, a)
        assert (a[0]["last"] >= 0).all() and float(a[2].item()) > 0


def test_noalloc_rejects_a_plan_beyond_the_scratch(gsr_lib):
    gsr = gsr_lib
    r = gsr.Renderer(0)
    cam = W.camera_replica()
    need = r.plan(400_000, [(cam.width, cam.height)], workspace=False)
    assert need > gsr.GSR_NOALLOC_SCRATCH_BYTES
    sc = W.random_scene(16, seed=0)  # arrays for the argument checks only; no launch happens
    g = gpu_scene(gsr, sc)
    cams = gsr.pack_cameras([cam])
    P = cam.width * cam.height
    tg = [torch.zeros(3 * P, device="cuda"), torch.zeros(P, device="cuda"), None]
    with pytest.raises(gsr.GsrError) as e:
        r.render_l1_fused_noalloc(g, cams, gsr.Config(flags=FLAGS_ALL), *tg, grads=r.new_grads(16))
    assert e.value.status == gsr.GSR_E_INVALID
    assert "static scratch" in str(e.value)
