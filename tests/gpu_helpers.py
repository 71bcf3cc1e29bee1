"""Helpers shared by the GPU parity tests: move seeded inputs to the device,
run the renderer through the C ABI, and compare with the CPU oracle."""
import numpy as np
import torch

import oracle as O


def gpu_scene(gsr, scene, mask=None):
    return gsr.Gaussians.from_arrays(scene.mean, scene.log_scale, scene.quat, scene.opacity_logit, scene.rgb,
                                     mask=mask)


def oracle_cfg_of(cfg):
    return O.Config(alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max, T_min=cfg.T_min, cutoff=cfg.cutoff_sigma,
                    z_near=cfg.z_near, lowpass=cfg.lowpass, bg=tuple(cfg.bg),
                    full_rect=bool(cfg.flags & 1))


def split_images(out, sizes):
    """Flat GPU outputs -> per-view numpy dicts (rgb [3,H,W], depth, T_final, last)."""
    res, po = [], 0
    rgb = out["rgb"].cpu().numpy()
    dep = out["depth"].cpu().numpy()
    T = out["T_final"].cpu().numpy()
    last = out["last"].cpu().numpy() if out.get("last") is not None else None
    for w, h in sizes:
        n = w * h
        res.append(dict(rgb=rgb[3 * po:3 * po + 3 * n].reshape(3, h, w), depth=dep[po:po + n].reshape(h, w),
                        T_final=T[po:po + n].reshape(h, w),
                        last=None if last is None else last[po:po + n].reshape(h, w)))
        po += n
    return res


def assert_images_close(gpu, orc, tol=1e-4, max_ambiguous=5e-3, check_last=True, done=None):
    """Colour, depth and transmittance within `tol` absolute and `last` exact
    on every pixel whose threshold decisions are unambiguous."""
    ok = ~orc["ambiguous"]
    if done is not None:
        ok &= done
        assert done.any()
    frac = 1.0 - ok.sum() / (done.sum() if done is not None else ok.size)
    amb = ~ok if done is None else (~ok & done)
    if amb.any():
        d_amb = np.maximum(np.abs(gpu["rgb"] - orc["rgb"]).max(0), np.abs(gpu["depth"] - orc["depth"]))[amb]
        print(f"ambiguous pixels: {int(amb.sum())} ({frac:.4%}); of these within tol: "
              f"{int((d_amb <= tol).sum())}", flush=True)
    assert frac <= max_ambiguous, f"ambiguous fraction {frac}"
    for k in ("depth", "T_final"):
        d = np.abs(gpu[k] - orc[k])[ok]
        assert d.size == 0 or d.max() <= tol, (k, float(d.max()), np.argwhere(np.abs(gpu[k] - orc[k]) * ok > tol)[:5])
    d = np.abs(gpu["rgb"] - orc["rgb"])[:, ok]
    assert d.size == 0 or d.max() <= tol, ("rgb", float(d.max()))
    if check_last:
        mism = (gpu["last"] != orc["last"]) & ok
        assert not mism.any(), ("last", np.argwhere(mism)[:5], gpu["last"][mism][:5], orc["last"][mism][:5])


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_grads_close(gpu, ref, rtol=1e-3, names=("mean", "log_scale", "quat", "opacity_logit", "rgb")):
    """Per tensor: ||g - g_ref|| <= rtol ||g_ref||; per element:
    |g - g_ref| <= rtol |g_ref| + rtol * rms(g_ref)."""
    for k in names:
        a = np.asarray(gpu[k], np.float64).reshape(-1)
        b = np.asarray(ref[k], np.float64).reshape(-1)
        e = rel_err(a, b)
        assert e <= rtol, (k, e)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        bad = np.abs(a - b) > rtol * np.abs(b) + rtol * rms
        assert not bad.any(), (k, np.argwhere(bad)[:5].ravel(), a[bad][:5], b[bad][:5])


def gpu_grads_numpy(gr):
    return dict(mean=gr["d_mean"].cpu().numpy(), log_scale=gr["d_log_scale"].cpu().numpy(),
                quat=gr["d_quat"].cpu().numpy(), opacity_logit=gr["d_opacity_logit"].cpu().numpy(),
                rgb=gr["d_rgb"].cpu().numpy(), pose=gr["d_pose"].cpu().numpy())


def flat_upstream(sizes, seed=1, zero_masks=None):
    """Generator upstream gradients as flat float32 tensors; pixels flagged in
    zero_masks (per view [H,W] bool) get zero upstream on every channel."""
    import workloads as W
    g_rgb, g_d, g_T = W.upstream_grads(sizes, seed=seed)
    if zero_masks is not None:
        po = 0
        for (w, h), m in zip(sizes, zero_masks):
            n = w * h
            mm = m.reshape(-1)
            for c in range(3):
                g_rgb[3 * po + c * n:3 * po + (c + 1) * n][mm] = 0.0
            g_d[po:po + n][mm] = 0.0
            g_T[po:po + n][mm] = 0.0
            po += n
    return g_rgb, g_d, g_T


def view_slices(flat_rgb, flat_d, flat_T, sizes):
    out, po = [], 0
    for w, h in sizes:
        n = w * h
        out.append((flat_rgb[3 * po:3 * po + 3 * n].reshape(3, h, w), flat_d[po:po + n].reshape(h, w),
                    flat_T[po:po + n].reshape(h, w)))
        po += n
    return out


def to_dev(x, dtype=torch.float32):
    return torch.as_tensor(x).to(device="cuda", dtype=dtype).contiguous()


def assert_close_scaled(a, b, rtol=1e-3, scale_tol=5e-4, what=""):
    """Element-wise |a - b| <= rtol |b| + scale_tol max|b|: for comparing two
    float32 results whose only difference is the order of atomic additions
    (sums with heavy cancellation lose digits relative to the tensor's scale,
    not to the element)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    m = np.abs(b).max() if b.size else 0.0
    bad = np.abs(a - b) > rtol * np.abs(b) + scale_tol * m
    assert not bad.any(), (what, int(bad.sum()), a[bad][:5], b[bad][:5], m)


def rect_pairs(proj):
    """Pairs the renderer emits: every tile of every valid Gaussian's
    rectangle (the lists then skip the tiles outside its alpha support)."""
    r = proj["rect"][proj["valid"]]
    return int(((r[:, 1] - r[:, 0] + 1) * (r[:, 3] - r[:, 2] + 1)).sum())


def oracle_work(o, cam, cfg_o):
    """Work totals of the oracle render `o` (from O.render) in the renderer's
    definitions: entries examined per pixel up to and including the one that
    stopped it, entries blended, and the sum of `last`; plus the summed list
    length of pixels with an ambiguous threshold decision (the most their
    counts can differ by)."""
    from oracle import splat as OS
    proj = o["proj"]
    starts, gauss = o["lists"]
    cfg = cfg_o.as_f32()
    TX = proj["TX"]
    evals = blended = slack = 0
    for tile in range(TX * proj["TY"]):
        px, py = OS._tile_pixels(tile, TX, int(cam.width), int(cam.height))
        lst = gauss[starts[tile]:starts[tile + 1]]
        L = lst.size
        if L == 0:
            continue
        r = OS._blend_tile(proj, lst, px, py, cfg)
        gate = r["alpha"] >= cfg.alpha_min
        P = np.cumprod(1.0 - np.where(gate, r["alpha"], 0.0), axis=1)
        stop = gate & (P < cfg.T_min)
        s = np.where(stop.any(axis=1), np.argmax(stop, axis=1) + 1, L)
        evals += int(s.sum())
        blended += int(r["contrib"].sum())
        slack += int(L * r["amb"].sum())
    return dict(fwd_evals=evals, blended=blended, bwd_evals=int(o["last"].sum()), slack=slack)
