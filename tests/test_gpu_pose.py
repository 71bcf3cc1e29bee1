"""Pose entry points through the C ABI against the oracle: cameras at
Exp(xi) T0 and from the paper's quaternion + translation, the xi gradient
J_l(xi)^T g, and the (q, t) gradient of a render (exact and
paper-approximate) at 1e-3."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

# rotation angles across the closed forms' series branch (|phi| < 1e-2) and beyond
XI = np.array([[0.0] * 6,
               [0.1, -0.2, 0.3, 0.0, 0.0, 0.0],
               [0.02, 0.01, -0.03, 1e-9, -2e-9, 1e-9],
               [0.5, -0.3, 0.2, 3e-3, -4e-3, 5e-3],
               [0.2, 0.4, -0.1, 0.005, 0.0, -0.0085],
               [0.3, -0.2, 0.1, 0.2, -0.3, 0.25],
               [-1.0, 0.5, 2.0, 1.2, 0.8, -1.9]])


def _cams(n):
    base = W.camera_small()
    out = []
    for v in range(n):
        c = W.perturb_pose(base, [0.1 * v, -0.05 * v, 0.2, 0.1 * v, 0.3, -0.2 * v])
        out.append(dataclasses.replace(c, R=c.R.astype(np.float32), t=c.t.astype(np.float32)))
    return out


def test_pose_apply_and_xi_gradient(gsr_lib):
    gsr = gsr_lib
    r = gsr.Renderer()
    cams0 = _cams(len(XI))
    c0 = gsr.pack_cameras(cams0)
    xi = XI.astype(np.float32)
    out = r.pose_apply(H.to_dev(xi), c0).cpu().numpy()
    for v, c in enumerate(cams0):
        R, t = O.apply_xi(xi[v].astype(np.float64), np.asarray(c.R, np.float64), np.asarray(c.t, np.float64))
        np.testing.assert_allclose(out[v, 4:13].reshape(3, 3), R, rtol=0, atol=1e-6, err_msg=str(v))
        np.testing.assert_allclose(out[v, 13:16], t, rtol=1e-6, atol=1e-6, err_msg=str(v))
        # intrinsics and size unchanged
        np.testing.assert_array_equal(out[v, :4], c0[v, :4].cpu().numpy())
        np.testing.assert_array_equal(out[v, 16:].view(np.int32), c0[v, 16:].cpu().numpy().view(np.int32))
    # Exp(0) leaves the pose bit for bit
    np.testing.assert_array_equal(out[0], c0[0].cpu().numpy())
    g = np.random.default_rng(0).normal(size=(len(XI), 6)).astype(np.float32)
    d_xi = r.pose_xi_grad(H.to_dev(xi), H.to_dev(g)).cpu().numpy()
    for v in range(len(XI)):
        want = O.pose_xi_grad(xi[v].astype(np.float64), g[v].astype(np.float64))
        np.testing.assert_allclose(d_xi[v], want, rtol=1e-5, atol=1e-6 * np.abs(want).max(), err_msg=str(v))
    np.testing.assert_array_equal(d_xi[0], g[0])  # J_l(0) = I


def _qt():
    q = np.array([[0.98, 0.05, -0.12, 0.1], [0.3, -0.9, 0.2, 0.25], [1.0, 0.0, 0.0, 0.0]], np.float32) * 1.3
    t = np.array([[0.03, -0.05, 0.08], [0.1, 0.2, -0.3], [0.0, 0.0, 0.0]], np.float32)
    return q, t


def test_pose_from_quaternion_translation(gsr_lib):
    gsr = gsr_lib
    r = gsr.Renderer()
    q, t = _qt()
    c0 = gsr.pack_cameras([W.camera_small()] * 3)
    out = r.pose_from_qt(H.to_dev(q), H.to_dev(t), c0).cpu().numpy()
    for v in range(3):
        R, tt = O.pose_from_qt(q[v].astype(np.float64), t[v].astype(np.float64))
        np.testing.assert_allclose(out[v, 4:13].reshape(3, 3), R, atol=1e-7)
        np.testing.assert_array_equal(out[v, 13:16], t[v])


@pytest.mark.parametrize("approx", [False, True])
def test_quaternion_translation_gradient_of_a_render(gsr_lib, approx):
    """Render at the poses of (q, t), backward to the left-perturbation pose
    gradient, chain to (q, t) on the device; against the oracle's gradient
    summed per Gaussian through dX_c/dq (and the covariance unless approx)."""
    gsr = gsr_lib
    sc = W.random_scene(2000, seed=13, xy=1.2)
    q, t = _qt()
    tmpl = W.camera_small()
    r = gsr.Renderer()
    r.plan(sc.n, [(tmpl.width, tmpl.height)] * 3)
    cams_d = r.pose_from_qt(H.to_dev(q), H.to_dev(t), gsr.pack_cameras([tmpl] * 3))
    flags = gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | (gsr.GSR_PAPER_POSE_APPROX if approx else 0)
    cfg = gsr.Config(flags=flags)
    g = H.gpu_scene(gsr, sc)
    r.render_forward(g, cams_d, cfg)
    cams = []
    cd = cams_d.cpu().numpy()
    for v in range(3):
        cams.append(dataclasses.replace(tmpl, R=cd[v, 4:13].reshape(3, 3).copy(), t=cd[v, 13:16].copy()))
    fwds = [O.render(sc, c) for c in cams]
    sizes = [(tmpl.width, tmpl.height)] * 3
    gr, gd, gT = H.flat_upstream(sizes, seed=4, zero_masks=[f["ambiguous_grad"] for f in fwds])
    grads = r.render_backward(g, cams_d, cfg, H.to_dev(gr), H.to_dev(gd), H.to_dev(gT))
    d_q, d_t = r.pose_qt_grad(H.to_dev(q), H.to_dev(t), grads["d_pose"])
    d_q, d_t = d_q.cpu().numpy(), d_t.cpu().numpy()
    for v, (c, f) in enumerate(zip(cams, fwds)):
        ur, ud, uT = H.view_slices(gr, gd, gT, sizes)[v]
        b = O.render_backward(sc, c, O.Config(), ur, ud, uT, approx_pose=approx, fwd=f)
        bq = O.backward_params(f["proj"], b["grad2d"], O.Config().as_f32(), approx_pose=approx,
                               pose_q=q[v].astype(np.float64))
        assert H.rel_err(d_q[v], bq["pose_q"]) <= 1e-3, (v, d_q[v], bq["pose_q"])
        assert H.rel_err(d_t[v], bq["pose_t"]) <= 1e-3, (v, d_t[v], bq["pose_t"])
