"""Helpers shared by the GPU parity tests: move seeded inputs to the device,
run the renderer through the C ABI, and compare with the CPU oracle."""
import numpy as np
import torch

import oracle as O


def gpu_scene(gsr, scene, mask=None):
    sh = getattr(scene, "sh", None)
    return gsr.Gaussians.from_arrays(scene.mean, scene.log_scale, scene.quat, scene.opacity_logit,
                                     scene.rgb if sh is None else None, mask=mask, sh=sh)


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


def last_ids(last, ranges, ids, tile_off, id_off, TX):
    """The Gaussian each pixel blended last (-1 where none), from a `last`
    image (1 + list position) and the tile lists it indexes: ranges [T, 2]
    and ids as the renderer's debug_tiles gives them (tile_off = the view's
    first tile, id_off = its first record id), or the oracle's
    (starts, gauss) as ranges = stack(starts[:-1], starts[1:])."""
    last = np.asarray(last)
    Hh, Ww = last.shape
    py, px = np.mgrid[0:Hh, 0:Ww]
    tile = (py // 16) * TX + px // 16
    base = np.asarray(ranges)[tile_off + tile, 0]
    pos = np.where(last > 0, base + last - 1, 0)
    ids = np.asarray(ids)
    got = ids[pos].astype(np.int64) - id_off if ids.size else np.zeros_like(pos)
    return np.where(last > 0, got, -1)


def gpu_view_lists(ranges, ids, tile_off, n_tiles, id_off):
    """One view's renderer lists in the oracle's (starts, gauss) form."""
    r = np.asarray(ranges)[tile_off:tile_off + n_tiles]
    a0 = int(r[0, 0]) if n_tiles else 0
    starts = np.concatenate([r[:, 0], r[-1:, 1]]) - a0 if n_tiles else np.zeros(1, np.int64)
    end = int(r[-1, 1]) if n_tiles else 0
    return starts.astype(np.int64), np.asarray(ids)[a0:end].astype(np.int64) - id_off


def oracle_ranges(lists):
    starts, _ = lists
    return np.stack([starts[:-1], starts[1:]], axis=1)


def assert_images_close(gpu, orc, tol=1e-4, max_ambiguous=5e-3, check_last=True, done=None, gpu_lists=None):
    """Colour, depth and transmittance within `tol` absolute, and the same
    last-blended Gaussian per pixel, on every pixel whose threshold decisions
    are unambiguous.  `last` is a position in a tile list and the renderer's
    lists leave out Gaussians that no pixel of the tile blends, so the
    positions are compared through the Gaussian they name: gpu_lists =
    (ranges, ids, tile_off, id_off) of the renderer's debug_tiles."""
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
        assert gpu_lists is not None, "comparing `last` needs the renderer's tile lists"
        TX = orc["proj"]["TX"]
        g_id = last_ids(gpu["last"], *gpu_lists, TX)
        o_id = last_ids(orc["last"], oracle_ranges(orc["lists"]), orc["lists"][1], 0, 0, TX)
        mism = (g_id != o_id) & ok
        assert not mism.any(), ("last", np.argwhere(mism)[:5], g_id[mism][:5], o_id[mism][:5])


def check_view_lists(ranges, ids, tile_off, id_off, proj, lists, width, height, cfg_o, tiles=None,
                     max_ambiguous=1e-4):
    """A view's tile lists against the oracle's (every Gaussian in every tile
    of its 3-sigma rectangle, ordered by float32 depth bits and index).  Per
    tile the renderer's list must be an in-order subsequence of the oracle's
    that keeps every Gaussian reaching alpha >= alpha_min at a pixel centre
    of the tile inside the image (FP64, every pixel) -- so each Gaussian it
    leaves out stays below alpha_min there and no pixel would blend it.
    Gaussians whose largest alpha lies within the float32 margin of
    alpha_min are counted as ambiguous (either choice is accepted) and their
    number is bounded.  Returns (oracle pairs, listed pairs, ambiguous)."""
    starts, gauss = lists
    cfg = cfg_o.as_f32()
    ranges = np.asarray(ranges)
    ids = np.asarray(ids)
    n_or = n_gpu = n_amb = 0
    for t in (range(proj["TX"] * proj["TY"]) if tiles is None else tiles):
        a, b = ranges[tile_off + t]
        got = ids[a:b].astype(np.int64) - id_off
        want = gauss[starts[t]:starts[t + 1]]
        n_or += want.size
        n_gpu += got.size
        order = np.argsort(want, kind="stable")
        k = np.searchsorted(want[order], got)
        assert np.all(k < want.size), ("renderer lists a Gaussian outside the rectangle lists", t)
        pos = order[k]
        assert np.array_equal(want[pos], got), ("renderer lists a Gaussian outside the rectangle lists", t)
        assert np.all(np.diff(pos) > 0), ("renderer list is not in (depth, index) order", t)
        amax = O.tile_alpha_max(proj, t, want, width, height, cfg)
        listed = np.zeros(want.size, bool)
        listed[pos] = True
        near = np.abs(amax - cfg.alpha_min) <= O.AMBIG_ALPHA * cfg.alpha_min
        missing = (amax >= cfg.alpha_min) & ~near & ~listed
        assert not missing.any(), ("renderer dropped a Gaussian that reaches alpha_min in the tile", t,
                                   want[missing][:5], amax[missing][:5])
        n_amb += int((near & ~listed).sum())
    assert n_amb <= max_ambiguous * max(n_or, 1), ("ambiguous drops", n_amb, n_or)
    return n_or, n_gpu, n_amb


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
    out = dict(mean=gr["d_mean"].cpu().numpy(), log_scale=gr["d_log_scale"].cpu().numpy(),
               quat=gr["d_quat"].cpu().numpy(), opacity_logit=gr["d_opacity_logit"].cpu().numpy(),
               pose=gr["d_pose"].cpu().numpy())
    if gr.get("d_rgb") is not None:
        out["rgb"] = gr["d_rgb"].cpu().numpy()
    if gr.get("d_sh") is not None:
        out["sh"] = gr["d_sh"].cpu().numpy()
    return out


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


def assert_close_scaled(a, b, rtol=1e-3, scale_tol=1e-4, what=""):
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


def oracle_work(o, cam, cfg_o, lists):
    """Work totals of the walk of `lists` (the renderer's own lists of this
    view as (starts, gauss)) with the oracle's arithmetic, in the renderer's
    definitions: entries examined per pixel up to and including the one that
    stopped it, entries blended, and the sum of `last`; plus the summed list
    length of pixels with an ambiguous threshold decision (the most their
    counts can differ by).  `o` is the oracle render of the view."""
    from oracle import splat as OS
    proj = o["proj"]
    starts, gauss = lists
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
    return dict(fwd_evals=evals, blended=blended, slack=slack)
