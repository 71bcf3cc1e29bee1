#!/usr/bin/env python3
"""Benchmark of the splatting renderer's training step on one MI355X.

Headline: forward + L1 loss + backward (all Gaussian parameters and the se(3)
pose) of 300k Gaussians at 1200x680 in a room-shaped synthetic scene,
reported as Mpixel/s.  One step = one launch of the HIP graph that holds the
whole fused step (projection, depth sort, pair emission, tile sort, ranges,
persistent forward/L1/backward rasteriser, chain to parameters and pose),
plus zeroing the gradient buffers.  Also reported: per-stage times and the
roofline of the dominant kernel (from an eager, event-timed loop of the same
step), the backward composite's algorithmic bytes against the copy-measured
achievable HBM bandwidth, the batched 16-keyframe launch against 16
per-frame launches, 72 pose hypotheses in one launch against 72 calls, the
coarse-to-fine tracking driver, and the CPU oracle timed on a bounded sample
of the same workloads (one process and forked worker processes).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpixel/s at 1200×680, 300k Gaussians; batched vs per-frame speedup"

# Algorithmic FP32 operations of the rasteriser, the per-unit figures of the
# method's cost model: about 20 per forward evaluation of one list entry at
# one pixel (Eq. 4-5: the conic quadratic form, opacity, blend) and about 70
# per backward evaluation (Eq. 11 and the supplement's blend gradient).  These
# make `roofline.achieved`.
FLOP_PER_FWD_EVAL, FLOP_PER_BWD_EVAL = 20, 70
# A finer count of the same work from the formulas (an FMA counts 2, exp2 /
# rcp count 1), reported beside it as `flop_per_launch_counted`:
#   forward evaluation of one list entry at one pixel: offset (2), quadratic
#     form (7), exp2 (1), opacity product (1), clamp (1), alpha test (1)   = 13
#   blending an accepted entry: 1 - alpha, T update, T test, weight, 4 FMAs = 12
#   backward re-evaluation of an entry (same as forward)                   = 13
#   backward contribution of an accepted entry: T recovery (2), weight (1),
#     colour/depth grads (4), dL/dalpha (17), running sums (12), clamp test
#     and scale (2), centre and conic grads (14), opacity grad (1), block
#     reduction adds for the 10 gradient fields (10)                      = 63
#   (the per-entry sums over the tile's pixels run as a matrix-core
#   contraction; they are counted at this algorithmic rate all the same).
FLOP_FWD_EVAL, FLOP_BLEND, FLOP_BWD_EVAL, FLOP_BWD_CONTRIB = 13, 12, 13, 63
# MI355X FP32 vector peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes
# x 2 (FMA) x 2.4 GHz.
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(batch):
    """HBM bytes per k_render_fused launch on the headline workload from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by the copy
    calibration), or None when the kernel sources changed since or the
    counters were taken on another staged batch size (another instantiation
    of the kernel) than `batch`."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_render_fused_traffic.json")
    try:
        rec = json.load(open(path))["records"][str(batch)]
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])
    except (OSError, ValueError, KeyError, TypeError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256") or rec.get("batch") != batch:
        return None
    return rec


def build_c2(gsr, torch, W, O=None):
    scene = W.room_scene(300_000, seed=0)
    cam = W.camera_replica()
    return scene, cam


def make_targets(gsr, torch, W, r, g, cams_d, sizes, seed=1):
    """Targets rendered from the scene itself plus 5% noise (depth noise is
    multiplicative; depth 0 where the accumulated opacity is below 0.5)."""
    out = r.render_forward(g, cams_d, gsr.Config())
    torch.cuda.synchronize()
    rgb = out["rgb"].cpu().numpy()
    dep = out["depth"].cpu().numpy()
    alpha = 1.0 - out["T_final"].cpu().numpy()
    t_rgb, t_d = W.noisy_targets(rgb, dep, seed=seed, sigma=0.05, min_alpha=0.5, alpha=alpha)
    return (torch.as_tensor(t_rgb).cuda(), torch.as_tensor(t_d).cuda()), r.pair_count()


def time_graph(torch, r, steps, warmup, stream):
    # The captured step overwrites gradients and loss (GSR_GRAD_OVERWRITE).
    def step():
        r.graph_launch(stream=stream)

    with torch.cuda.stream(stream):
        for _ in range(warmup):
            step()
        stream.synchronize()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        e1.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, wall


def run_headline(args, gsr, torch, W):
    scene, cam = build_c2(gsr, torch, W)
    sizes = [(cam.width, cam.height)]
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    cams_d = gsr.pack_cameras([cam])
    r = gsr.Renderer(0)
    r.plan(scene.n, sizes)
    (t_rgb, t_d), pairs = make_targets(gsr, torch, W, r, g, cams_d, sizes)
    r.plan(scene.n, sizes, pair_capacity=int(pairs * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    tuning = r.get_tuning()
    if args.tuning:
        vals = [int(x) for x in args.tuning.split(",")]
        b, p, l = vals[:3]
        r.set_tuning(blocks_per_cu=b, tiles_per_pop=p, lpt_order=l, batch=vals[3] if len(vals) > 3 else 192)
        tuning = r.get_tuning()
        log("tuning:", tuning)
    elif not args.no_autotune:
        tuning = r.autotune(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, reps=2)
        log("autotune:", tuning)
    grads = r.new_grads(scene.n)
    loss = torch.zeros(1, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss, stream=stream)
    stream.synchronize()
    ms, wall = time_graph(torch, r, args.steps, args.warmup, stream)
    r.check_overflow(stream=stream)
    log(f"graph step: {ms:.3f} ms (wall {wall:.3f} ms), loss {loss.item():.2f}")

    # Eager, event-timed loop of the same step for per-stage times.
    r.set_profiling(True)
    for _ in range(3):
        r.render_l1_fused(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss)
    r.stage_times()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        r.render_l1_fused(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss)
    e1.record()
    e1.synchronize()
    eager_ms = e0.elapsed_time(e1) / args.steps
    st = r.stage_times()
    r.set_profiling(False)
    calls = max(1, st.pop("calls"))
    stages = {k: v / calls for k, v in st.items()}
    work = r.work_counts(g, cfg)
    rng, _ = r.debug_tiles()
    # pairs inside the tile lists (the rest lie outside their Gaussian's alpha support)
    work["pairs_listed"] = int((rng[:, 1] - rng[:, 0]).clamp(min=0).sum())
    raster_ms = stages["raster"]
    flops = work["fwd_evals"] * FLOP_PER_FWD_EVAL + work["bwd_evals"] * FLOP_PER_BWD_EVAL
    counted = (work["fwd_evals"] * FLOP_FWD_EVAL + work["blended"] * FLOP_BLEND +
               work["bwd_evals"] * FLOP_BWD_EVAL + work["blended"] * FLOP_BWD_CONTRIB)
    achieved = flops / (raster_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 1),
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": "k_render_fused", "kernel_ms": round(raster_ms, 4), "flop_per_launch": int(flops),
            "flop_per_launch_counted": int(counted),
            "frac_counted": round(counted / (raster_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
    tr = measured_traffic(tuning.get("batch"))
    if tr is not None:
        # bytes per launch, HBM read + written (rocprofv3 counters, copy-calibrated)
        roof["traffic"] = int(tr["bytes_total"])
        roof["traffic_read"] = int(tr["bytes_read"])
        roof["traffic_written"] = int(tr["bytes_written"])
        roof["traffic_source"] = tr["summary"]
    px = cam.width * cam.height
    roof["a7_backward_hbm"] = backward_hbm(args, gsr, torch, r, g, cams_d, cam, t_rgb, t_d, raster_ms, work)
    if tr is not None and tr.get("valu_busy") is not None:
        roof["valu_busy"] = tr["valu_busy"]
    return dict(ms=ms, wall=wall, eager_ms=eager_ms, stages=stages, work=work, roof=roof, tuning=tuning,
                mpx=px / (ms * 1e-3) / 1e6, pairs=pairs)


def achievable_hbm_gbs(torch, mib=1024, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of `mib` MiB (read +
    write bytes over its event-timed duration, best of `reps`)."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def visited_pairs(torch, last, width, height):
    """P_v: the sum over tiles of the tile's longest walked list prefix (the
    largest `last` of its pixels)."""
    TX, TY = (width + 15) // 16, (height + 15) // 16
    img = torch.zeros(TY * 16, TX * 16, dtype=torch.int32, device=last.device)
    img[:height, :width] = last.view(height, width)
    return int(img.view(TY, 16, TX, 16).amax(dim=(1, 3)).to(torch.int64).sum().item())


def backward_hbm(args, gsr, torch, r, g, cams_d, cam, t_rgb, t_d, fused_ms, work):
    """The backward composite (A7) against HBM bandwidth: algorithmic bytes
    P_v x (4 B list id + 40 B record + 40 B gradient atomics) + pixels x
    (8 B saved state + 16 B upstream gradient), over the standalone backward
    kernel's time (forward, L1 gradient and backward as separate calls, the
    backward stage event-timed) and over the fused kernel's time, as
    fractions of the copy-measured achievable bandwidth.  Also the
    backward's ALU floor: its algorithmic FLOPs at the FP32 vector peak, and
    the bandwidth fraction the byte model would reach even at that floor."""
    px = cam.width * cam.height
    cfg = gsr.Config()
    out = r.new_images()
    r.set_profiling(True)
    for it in range(3 + args.steps):
        if it == 3:
            r.stage_times()
        r.render_forward(g, cams_d, cfg, out=out, check=False)
        _, gC, gD = r.l1_loss_grad(out["rgb"], out["depth"], t_rgb, t_d, None, 1.0, 0.1)
        r.render_backward(g, cams_d, cfg, gC, gD, None)
    st = r.stage_times()
    r.set_profiling(False)
    r.check_overflow()
    bwd_ms = st["raster_bwd"] / args.steps  # (the forward calls are timed calls too)
    pv = visited_pairs(torch, out["last"], cam.width, cam.height)
    bytes_alg = pv * 84 + px * 24
    ach = achievable_hbm_gbs(torch)
    gbs_b = bytes_alg / (bwd_ms * 1e-3) / 1e9
    gbs_f = bytes_alg / (fused_ms * 1e-3) / 1e9
    bwd_flop = work["bwd_evals"] * FLOP_PER_BWD_EVAL
    floor_ms = bwd_flop / (PEAK_FP32_TFLOPS * 1e12) * 1e3
    return {"kernel": "k_render_bwd", "visited_pairs": pv, "bytes_alg": int(bytes_alg),
            "bwd_flop": int(bwd_flop), "alu_frac": round(bwd_flop / (bwd_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "alu_floor_ms": round(floor_ms, 4),
            "frac_of_achievable_at_alu_floor": round(bytes_alg / (floor_ms * 1e-3) / 1e9 / ach, 4),
            "kernel_ms": round(bwd_ms, 4), "achieved_gbs": round(gbs_b, 1), "achievable_gbs": round(ach, 1),
            "frac_of_achievable": round(gbs_b / ach, 4), "frac_of_peak": round(gbs_b / 8000.0, 4),
            "fused_kernel_gbs": round(gbs_f, 1), "fused_frac_of_achievable": round(gbs_f / ach, 4),
            "target_frac": 0.5, "met": bool(gbs_b / ach >= 0.5), **backward_counters(bytes_alg, bwd_ms, ach)}


def backward_counters(bytes_alg, bwd_ms, ach):
    """The standalone backward kernel's HBM bytes from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record (copy-calibrated) and its VALU-busy
    fraction (SQ_INSTS_VALU x 4 cycles over its SIMD-cycles), while its
    sources are unchanged; the counter bytes are flagged when they exceed
    1.5x the byte model."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_render_fused_traffic.json")
    try:
        rec = json.load(open(path))["k_render_bwd"]
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])
    except (OSError, ValueError, KeyError, TypeError):
        return {"counter_bytes": None}
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return {"counter_bytes": None}
    cb = int(rec["bytes_total"])
    gbs = cb / (bwd_ms * 1e-3) / 1e9
    return {"counter_bytes": cb, "counter_gbs": round(gbs, 1), "counter_frac_of_achievable": round(gbs / ach, 4),
            "counter_over_alg": round(cb / bytes_alg, 3), "counter_flag": bool(cb > 1.5 * bytes_alg),
            "valu_busy": rec.get("valu_busy"), "counter_source": rec["summary"]}


def run_sh(args, gsr, torch, W, tuning):
    """The headline step with degree-1 spherical-harmonic colour (12
    coefficients per Gaussian, Sec. 3.1) in place of RGB: the same scene
    with seeded coefficients, graph-captured, at the headline's tuning; the
    projection evaluates the colour per view and the chain carries its
    gradient to the coefficients, the mean and the pose."""
    scene, cam = build_c2(gsr, torch, W)
    sc = W.with_sh(scene)
    sizes = [(cam.width, cam.height)]
    g = gsr.Gaussians.from_arrays(sc.mean, sc.log_scale, sc.quat, sc.opacity_logit, None, sh=sc.sh)
    cams_d = gsr.pack_cameras([cam])
    r = gsr.Renderer(0)
    r.plan(sc.n, sizes)
    (t_rgb, t_d), pairs = make_targets(gsr, torch, W, r, g, cams_d, sizes)
    r.plan(sc.n, sizes, pair_capacity=int(pairs * 1.25) + 4096)
    r.set_tuning(**tuning)
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    grads = r.new_grads(sc.n, sh=True)
    loss = torch.zeros(1, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss, stream=stream)
    stream.synchronize()
    ms, _ = time_graph(torch, r, args.steps, args.warmup, stream)
    r.check_overflow(stream=stream)
    r.set_profiling(True)
    for _ in range(3):
        r.render_l1_fused(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss)
    r.stage_times()
    for _ in range(args.steps):
        r.render_l1_fused(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss)
    st = r.stage_times()
    r.set_profiling(False)
    calls = max(1, st.pop("calls"))
    return {"workload": "the headline step (300k Gaussians, 1200x680, fwd+L1+bwd) with degree-1 SH colour",
            "ms_per_step": round(ms, 4), "mpx_s": round(cam.width * cam.height / (ms * 1e-3) / 1e6, 1),
            "stages_ms": {k: round(v / calls, 4) for k, v in st.items()}}


def run_expansion(args, gsr, torch, W):
    """Map expansion (Sec. 3.2) on the headline workload: the adding step
    (Eq. 8) over the rendered 1200x680 keyframe against the room's observed
    depth, and the deleting step (Eq. 9) over the 300k Gaussians; each timed
    with events over `steps` calls, against HBM bandwidth with the
    algorithmic bytes: adding 12 B per pixel (T_final, rendered and observed
    depth) + per new Gaussian 16 B read (depth, colour) + 56 B written;
    deleting 12 + 4 B read, 4 B gather, 4 + 1 B written per Gaussian."""
    scene, cam = build_c2(gsr, torch, W)
    sizes = [(cam.width, cam.height)]
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    cams_d = gsr.pack_cameras([cam])
    r = gsr.Renderer(0)
    r.plan(scene.n, sizes)
    img = r.render_forward(g, cams_d, gsr.Config())
    obs = torch.as_tensor(W.room_depth(cam)).cuda()
    rgb_obs = torch.as_tensor(W.random_targets(sizes, seed=1)[0]).cuda()
    px = cam.width * cam.height
    cap = px
    z = lambda *sh: torch.empty(*sh, device="cuda")  # noqa: E731
    out = dict(mean=z(cap, 3), log_scale=z(cap, 3), quat=z(cap, 4), opacity_logit=z(cap), rgb=z(cap, 3))
    tau_T, tau_D = 0.5, 0.1
    count = torch.zeros(1, dtype=torch.int64, device="cuda")

    def add():
        r.expand_add(cams_d, img["T_final"], img["depth"], obs, rgb_obs, out, 0, cap, tau_T, tau_D, count=count)

    logit_out = z(scene.n)
    dec = torch.empty(scene.n, dtype=torch.uint8, device="cuda")

    def delete():
        r.expand_delete(g, cams_d, obs, cam.width, cam.height, 0.1, 0.01, logit_out=logit_out, decayed=dec)

    res = {}
    for name, fn in (("add", add), ("delete", delete)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        e1.synchronize()
        res[name] = e0.elapsed_time(e1) / args.steps
    added = int(count.item())
    decayed = int(dec.sum().item())
    b_add = px * 12 + added * (16 + 56)
    b_del = scene.n * (12 + 4 + 4 + 4 + 1)
    return {"workload": "adding step over one 1200x680 keyframe of the 300k-Gaussian room render (observed depth: "
                        "the room box, 5% missing; tau_T 0.5, tau_D 0.1 m); deleting step over the 300k Gaussians "
                        "(gamma 0.1 m, eta 0.01)",
            "add_ms": round(res["add"], 4), "added": added, "add_bytes_alg": int(b_add),
            "add_hbm_frac": round(b_add / (res["add"] * 1e-3) / 8e12, 4),
            "add_mpx_s": round(px / (res["add"] * 1e-3) / 1e6, 1),
            "delete_ms": round(res["delete"], 4), "decayed": decayed, "delete_bytes_alg": int(b_del),
            "delete_hbm_frac": round(b_del / (res["delete"] * 1e-3) / 8e12, 4)}


def run_batched(args, gsr, torch, W):
    """16 keyframes of mixed resolution over 1M Gaussians: one graph launch
    of the batched fused step vs 16 per-frame fused calls on the same stream
    (gradients accumulated into the same buffers)."""
    scene = W.room_scene(1_000_000, seed=0)
    cams = W.mapping_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    cams_d = gsr.pack_cameras(cams)
    rb = gsr.Renderer(0)
    rb.plan(scene.n, sizes)
    (t_rgb, t_d), pairs = make_targets(gsr, torch, W, rb, g, cams_d, sizes)
    rb.plan(scene.n, sizes, pair_capacity=int(pairs * 1.25) + 4096)
    cfg = gsr.Config(flags=gsr.GSR_GAUSS_GRAD | gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    if not args.no_autotune:
        rb.autotune(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, reps=2)
    grads = rb.new_grads(scene.n)
    loss = torch.zeros(1, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rb.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss, stream=stream)
    stream.synchronize()
    steps = max(3, args.steps // 4)
    b_ms, _ = time_graph(torch, rb, steps, 2, stream)
    rb.check_overflow(stream=stream)
    del rb
    torch.cuda.empty_cache()

    # Per-frame: one renderer per view (planned once), 16 calls per step.
    offs, po = [], 0
    for w, h in sizes:
        offs.append(po)
        po += w * h
    per = []
    for v, c in enumerate(cams):
        r = gsr.Renderer(0)
        w, h = sizes[v]
        r.plan(scene.n, [sizes[v]])
        tr = t_rgb[3 * offs[v]:3 * offs[v] + 3 * w * h]
        td = t_d[offs[v]:offs[v] + w * h]
        cd = gsr.pack_cameras([c])
        if not args.no_autotune:  # each per-frame renderer tuned on its own view
            r.autotune(g, cd, cfg, tr, td, None, 1.0, 0.1, reps=2)
        per.append((r, cd, tr, td))
    pose = torch.zeros(1, 6, device="cuda")
    gr1 = dict(grads)
    cfg_acc = gsr.Config()  # the frames add into the same buffers

    def step():
        for t in grads.values():
            t.zero_()
        loss.zero_()
        for v, (r, cd, tr, td) in enumerate(per):
            gr1["d_pose"] = grads["d_pose"][v:v + 1]
            r.render_l1_fused(g, cd, cfg_acc, tr, td, None, 1.0, 0.1, grads=gr1, loss=loss)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    e1.synchronize()
    p_ms = e0.elapsed_time(e1) / steps
    del per, pose
    torch.cuda.empty_cache()
    total_px = sum(w * h for w, h in sizes)
    return {"workload": "1M Gaussians, 16 keyframes (4x320x240, 8x640x480, 4x1200x680), fwd+L1+bwd",
            "batched_ms": round(b_ms, 3), "per_frame_ms": round(p_ms, 3),
            "speedup": round(p_ms / b_ms, 3), "batched_mpx_s": round(total_px / (b_ms * 1e-3) / 1e6, 1),
            "per_frame_mpx_s": round(total_px / (p_ms * 1e-3) / 1e6, 1), "pairs": int(pairs)}


def run_hypotheses(args, gsr, torch, W):
    """500k Gaussians, 64 pose hypotheses at 600x340 plus 8 at 1200x680 in one
    launch, forward + L1 + backward to the poses only: per-batch latency
    p50/p99 of the captured step against 72 separate per-pose calls."""
    import numpy as np
    scene = W.room_scene(500_000, seed=0)
    cams = W.hypothesis_views(seed=2)
    sizes = [(c.width, c.height) for c in cams]
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    base_full = W.camera_replica()
    h = W.camera_hyp_half()
    base_half = base_full.with_size(h.fx, h.fy, h.cx, h.cy, h.width, h.height)
    tg = {}
    for key, cam in (("half", base_half), ("full", base_full)):
        r = gsr.Renderer(0)
        r.plan(scene.n, [(cam.width, cam.height)])
        (trgb, td), _ = make_targets(gsr, torch, W, r, g, gsr.pack_cameras([cam]), [(cam.width, cam.height)])
        tg[key] = (trgb, td)
        del r
    t_rgb = torch.cat([tg["half" if w == 600 else "full"][0] for w, _ in sizes])
    t_d = torch.cat([tg["half" if w == 600 else "full"][1] for w, _ in sizes])
    cfg = gsr.Config(flags=gsr.GSR_POSE_GRAD | gsr.GSR_GRAD_OVERWRITE)
    cfg_acc = gsr.Config(flags=gsr.GSR_POSE_GRAD)
    cams_d = gsr.pack_cameras(cams)
    rb = gsr.Renderer(0)
    rb.plan(scene.n, sizes)
    rb.render_forward(g, cams_d, cfg)
    pairs = rb.pair_count()
    rb.plan(scene.n, sizes, pair_capacity=int(pairs * 1.25) + 4096)
    if not args.no_autotune:
        rb.autotune(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, reps=2)
    grads = {"d_pose": torch.zeros(len(cams), 6, device="cuda")}
    loss = torch.zeros(1, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rb.graph_capture(g, cams_d, cfg, t_rgb, t_d, None, 1.0, 0.1, grads=grads, loss=loss, stream=stream)
    stream.synchronize()
    lat = []
    with torch.cuda.stream(stream):
        for it in range(args.hyp_batches + 3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rb.graph_launch(stream=stream)
            e1.record(stream)
            e1.synchronize()
            if it >= 3:
                lat.append(e0.elapsed_time(e1))
    rb.check_overflow(stream=stream)
    del rb
    torch.cuda.empty_cache()
    lat = np.array(lat)
    # 72 separate calls: one renderer per resolution, reused view after view.
    rs = {}
    offs, po = [], 0
    for w, hh in sizes:
        offs.append(po)
        po += w * hh
    per_cams = [gsr.pack_cameras([c]) for c in cams]
    for key, cam in (("half", base_half), ("full", base_full)):
        r = gsr.Renderer(0)
        r.plan(scene.n, [(cam.width, cam.height)])
        if not args.no_autotune:  # tuned on the first hypothesis of its resolution
            v = next(k for k, (w, hh) in enumerate(sizes) if (w, hh) == (cam.width, cam.height))
            w, hh = sizes[v]
            r.autotune(g, per_cams[v], cfg_acc, t_rgb[3 * offs[v]:3 * (offs[v] + w * hh)],
                       t_d[offs[v]:offs[v] + w * hh], None, 1.0, 0.1, reps=2)
        rs[(cam.width, cam.height)] = r
    gr1 = {"d_pose": None}

    def step():
        grads["d_pose"].zero_()
        loss.zero_()
        for v, (w, hh) in enumerate(sizes):
            gr1["d_pose"] = grads["d_pose"][v:v + 1]
            rs[(w, hh)].render_l1_fused(g, per_cams[v], cfg_acc, t_rgb[3 * offs[v]:3 * (offs[v] + w * hh)],
                                        t_d[offs[v]:offs[v] + w * hh], None, 1.0, 0.1, grads=gr1, loss=loss)

    step()
    torch.cuda.synchronize()
    reps = max(3, args.hyp_batches // 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    e1.synchronize()
    sep_ms = e0.elapsed_time(e1) / reps
    del rs
    torch.cuda.empty_cache()
    total_px = sum(w * hh for w, hh in sizes)
    return {"workload": "500k Gaussians, 64 poses at 600x340 + 8 at 1200x680, fwd+L1+bwd to pose only",
            "batches": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "separate_ms": round(sep_ms, 3),
            "speedup": round(sep_ms / float(np.percentile(lat, 50)), 3),
            "batched_mpx_s": round(total_px / (float(np.percentile(lat, 50)) * 1e-3) / 1e6, 1),
            "pairs": int(pairs)}


def _track_once(gsr, torch, W, scene, truth, tc, render_mask=None):
    """One timed coarse-to-fine tracking run (after one warm-up run): targets
    rendered at `truth` (with `render_mask` selecting the Gaussians that
    appear in them), 10% of the depth readings removed, start perturbed by
    2 cm / 1 deg.  Returns the timing, the start and end pose errors and the
    fine stage's selected Gaussians."""
    import numpy as np
    from paper_2311_11700_amd.tracking import Tracker
    g = gsr.Gaussians.from_arrays(*scene.arrays())
    r = gsr.Renderer(0)
    r.plan(scene.n, [(truth.width, truth.height)])
    gm = g if render_mask is None else gsr.Gaussians(g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb,
                                                     render_mask)
    out = r.render_forward(gm, gsr.pack_cameras([truth]), gsr.Config())
    t_rgb, t_d = out["rgb"].clone(), out["depth"].clone()
    rng = np.random.default_rng(3)
    t_d[torch.as_tensor(rng.random(t_d.numel()) < 0.1, device="cuda")] = 0.0
    del r
    start = W.tracking_start(seed=2, truth=truth)
    T0 = np.eye(4)
    T0[:3, :3], T0[:3, 3] = start.R, start.t
    tr = Tracker(g, truth, tc)
    tr.track(torch.tensor(T0), t_rgb, t_d)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    T = tr.track(torch.tensor(T0), t_rgb, t_d)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    T = T.cpu().numpy()
    Tt = np.eye(4)
    Tt[:3, :3], Tt[:3, 3] = truth.R, truth.t
    E0, E1 = T0 @ np.linalg.inv(Tt), T @ np.linalg.inv(Tt)

    def ang(R):
        return float(np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))))

    iters = tc.coarse_iters + tc.fine_iters
    return {"reliable": int(tr.reliable.sum().item()),
            "ms_total": round(ms, 2), "ms_per_iter": round(ms / iters, 3),
            "trans_err_cm": [round(float(np.linalg.norm(E0[:3, 3])) * 100, 3),
                             round(float(np.linalg.norm(E1[:3, 3])) * 100, 3)],
            "rot_err_deg": [round(ang(E0[:3, :3]), 3), round(ang(E1[:3, :3]), 3)]}


def run_tracking(args, gsr, torch, W):
    """Coarse-to-fine tracking of one frame, 640x480 (coarse 160x120), 5 + 95
    pose-only iterations, start perturbed by 2 cm / 1 deg, 10% of the depth
    readings removed.  Two maps:
    - the configured one: the 150k-Gaussian room scene seen from the TUM
      camera at its identity pose, the fine stage on the Gaussians with
      sigmoid(opacity) > 0.5;
    - flat surface Gaussians of the room plus 5% outliers 0.3-0.6 m off the
      surfaces (the target rendered from the surfaces only), the fine stage on
      the Eq. 12 reliable Gaussians (eps 0.3 m), which must drop the
      outliers."""
    from paper_2311_11700_amd.tracking import TrackingConfig
    conf = _track_once(gsr, torch, W, W.room_scene(150_000, seed=0), W.camera_tum(),
                       TrackingConfig(reliable_eps=float("inf"), reliable_opacity=0.5))
    conf["workload"] = ("150k Gaussians (room scene), 640x480 TUM camera at its identity pose (coarse 160x120), "
                        "5 + 95 iterations, pose-only, fine stage on sigmoid(opacity) > 0.5")
    scene, n_surf = W.tracking_scene(150_000, seed=0, outlier_fraction=0.05, offset=(0.3, 0.6))
    surf = torch.zeros(scene.n, dtype=torch.uint8, device="cuda")
    surf[:n_surf] = 1
    res = _track_once(gsr, torch, W, scene, W.camera_tracking(), TrackingConfig(reliable_eps=0.3),
                      render_mask=surf)
    res["workload"] = ("150k Gaussians (flat surface Gaussians + 5% outliers), 640x480 (coarse 160x120), "
                       "5 + 95 iterations, pose-only, fine stage on Eq. 12 reliable Gaussians (eps 0.3 m)")
    res["configured_scene"] = conf
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


# State of the CPU-baseline sample, inherited by forked worker processes.
_CPU = {}


def _oracle_tiles(tiles):
    """Forward + L1 + backward of `tiles` of the prepared workload with the
    FP64 oracle, one thread; returns the pixels done."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    st = _CPU
    proj, (starts, gauss), cfg, cam = st["proj"], st["lists"], st["cfg"], st["cam"]
    px = 0
    with threadpool_limits(1):
        for tile in tiles:
            pxs, pys = O.splat._tile_pixels(tile, proj["TX"], cam.width, cam.height)
            lst = gauss[starts[tile]:starts[tile + 1]]
            rr = O.splat._blend_tile(proj, lst, pxs, pys, cfg)
            if st["backward"]:
                e = rr["C"].T - st["t_rgb"][:, pys, pxs]
                ed = rr["D"] - st["t_d"][pys, pxs]
                gC = np.sign(e).T
                gD = 0.1 * np.sign(ed) * (st["t_d"][pys, pxs] > 0)
                O.splat._blend_tile_backward(proj, lst, pxs, pys, cfg, rr, gC, gD, np.zeros_like(gD))
            px += pxs.size
    return px


def _oracle_frame(W, scene, cam, backward, budget_s, workers, seed=0):
    """Full-frame oracle time estimated from a sample: projection and tile
    lists of all Gaussians, then tiles in a seeded random order until
    `budget_s`, one process (and the same number of tiles per worker across
    `workers` forked processes), then the per-Gaussian chain of the whole
    frame (backward only).  Returns per-mode seconds for the whole frame."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    cfg = O.Config().as_f32()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        proj = O.project(scene, cam, cfg)
        lists = O.tile_lists(proj)
        t_geo = time.perf_counter() - t0
    T = proj["TX"] * proj["TY"]
    t_rgb, t_d, _ = W.random_targets([(cam.width, cam.height)], seed=1)
    _CPU.update(proj=proj, lists=lists, cfg=cfg, cam=cam, backward=backward,
                t_rgb=t_rgb.reshape(3, cam.height, cam.width), t_d=t_d.reshape(cam.height, cam.width))
    order = np.random.default_rng(seed).permutation(T)
    # one process: tiles in chunks of 8 until the budget
    t1 = time.perf_counter()
    done = 0
    while done < T and time.perf_counter() - t1 < budget_s:
        _oracle_tiles(order[done:done + 8])
        done += min(8, T - done)
    t_one = time.perf_counter() - t1
    t_chain = 0.0
    if backward:
        with threadpool_limits(1):
            t2 = time.perf_counter()
            O.backward_params(proj, np.zeros((proj["n"], 10)), cfg)
            t_chain = time.perf_counter() - t2
    one = t_geo + t_chain + t_one * T / done
    # `workers` processes: the next (workers x done) tiles, one chunk each
    multi, m_done = None, 0
    if workers > 1:
        m_tiles = np.concatenate([order[done:], order[:done]])[: min(T, workers * done)]
        chunks = [c for c in np.array_split(m_tiles, workers * 4) if c.size]
        with mp.get_context("fork").Pool(workers) as pool:
            t3 = time.perf_counter()
            pool.map(_oracle_tiles, chunks, chunksize=1)
            t_multi = time.perf_counter() - t3
        m_done = int(m_tiles.size)
        multi = t_geo + t_chain + t_multi * T / m_done
    _CPU.clear()
    return dict(tiles=T, sample_one=done, sample_multi=m_done, t_geo=t_geo, t_chain=t_chain, one=one, multi=multi)


def cpu_baseline(args, W):
    """The FP64 oracle as it stands on the host cores: the 300k-Gaussian
    1200x680 step (forward + L1 + backward) and the 2 000-Gaussian 160x120
    forward, each timed in one process and in `workers` forked processes over
    tile chunks, on a bounded sample of tiles scaled to the whole frame."""
    workers = max(1, min(16, os.cpu_count() or 1))
    budget = args.cpu_seconds
    scene, cam = W.room_scene(300_000, seed=0), W.camera_replica()
    c2 = _oracle_frame(W, scene, cam, True, 0.35 * budget, workers)
    px2 = cam.width * cam.height
    small, cam1 = W.random_scene(2000, seed=0), W.camera_small()
    c1 = _oracle_frame(W, small, cam1, False, 0.1 * budget, workers)
    px1 = cam1.width * cam1.height
    best = c2["multi"] if c2["multi"] else c2["one"]
    return {"value": round(px2 / best / 1e6, 6), "unit": "Mpixel/s", "cores": workers, "kind": "oracle",
            "sample": (f"300k-Gaussian 1200x680 step (forward + L1 + backward, FP64): {c2['sample_one']} of "
                       f"{c2['tiles']} tiles in one process, {c2['sample_multi']} over {workers} processes; "
                       f"projection and tile lists ({c2['t_geo']:.1f} s) and the per-Gaussian chain "
                       f"({c2['t_chain']:.1f} s) of the whole frame added once; scaled to the whole frame"),
            "value_1core": round(px2 / c2["one"] / 1e6, 6),
            "frame_seconds": {"multi": round(c2["multi"], 2) if c2["multi"] else None, "one": round(c2["one"], 2)},
            "small_forward": {"workload": "2 000 Gaussians, 160x120, forward only",
                              "mpx_s_multi": round(px1 / c1["multi"] / 1e6, 6) if c1["multi"] else None,
                              "mpx_s_1core": round(px1 / c1["one"] / 1e6, 6),
                              "sample_tiles": [c1["sample_one"], c1["sample_multi"], c1["tiles"]]},
            "cpu": cpu_model(), "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", type=str, default=None,
                    help="blocks_per_cu,tiles_per_pop,lpt_order[,batch] for the headline (skips its autotune)")
    ap.add_argument("--no-extra", action="store_true", help="skip the pose-hypothesis, tracking and SH-colour legs")
    ap.add_argument("--hyp-batches", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); the renderer has no "
              "multi-GPU path to time", file=sys.stderr)
        sys.exit(2)

    import workloads as W

    cpu = None
    if not args.no_cpu_baseline:
        # The oracle on the host cores, in forked worker processes: before
        # this process initialises the GPU.
        log("cpu baseline (oracle sample)")
        cpu = cpu_baseline(args, W)
        log("cpu:", cpu)

    import torch

    import paper_2311_11700_amd as gsr

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration_mb:
        nb = args.copy_calibration_mb << 20
        src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration_mb} MB")
        del src, dst
    log("headline: 300k Gaussians, 1200x680")
    h = run_headline(args, gsr, torch, W)
    log("map expansion: 300k Gaussians, 1200x680")
    expansion = run_expansion(args, gsr, torch, W)
    log("expansion:", expansion)
    sh_leg = None
    if not args.no_extra:
        log("SH colour: 300k Gaussians, 1200x680")
        sh_leg = run_sh(args, gsr, torch, W, h["tuning"])
        log("sh colour:", sh_leg)
    batched = None
    if not args.no_batched:
        log("batched: 1M Gaussians, 16 keyframes")
        batched = run_batched(args, gsr, torch, W)
        log("batched:", batched)
    hyp = trk = None
    if not args.no_extra:
        log("pose hypotheses: 500k Gaussians, 72 views")
        hyp = run_hypotheses(args, gsr, torch, W)
        log("hypotheses:", hyp)
        log("tracking: 150k Gaussians, 640x480")
        trk = run_tracking(args, gsr, torch, W)
        log("tracking:", trk)
    line = {
        "metric": METRIC,
        "value": round(h["mpx"], 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fwd+L1+bwd, 300k Gaussians (room scene, 70% on walls/floor), 1200x680, f=600; "
                               "grads to all Gaussian parameters and the se(3) pose; HIP graph of the fused step",
                   "gaussians": 300000, "width": 1200, "height": 680, "loss": "L1 rgb + 0.1 L1 depth"},
        "roofline": h["roof"],
        "cpu_baseline": cpu,
        "batched": batched,
        "hypotheses": hyp,
        "tracking": trk,
        "expansion": expansion,
        "sh_colour": sh_leg,
        "eager_ms_per_step": round(h["eager_ms"], 4),
        "stages_ms": {k: round(v, 4) for k, v in h["stages"].items()},
        "work": h["work"],
        "tuning": h["tuning"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
