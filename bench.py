#!/usr/bin/env python
"""Benchmark of the masked 4D Gaussian rasterizer on one MI355X.

Headline step: render one 1352x1014 frame of a 200k-Gaussian long-lifespan
scene (20 cameras on a 120-degree arc, 300 timestamps) through the whole
forward path: keyframe active set (one mask per 10-frame window, built before
timing) -> slice/project/shade -> visible compaction -> depth sort -> tile
keys -> tile sort -> ranges -> per-tile blending.  value = frames/s over
--steps frames, inputs resident in HBM, with consecutive frames dealt
round-robin over --streams streams (default 4, one context and one image
each, on eight hardware queues; the one-stream rate is reported beside it).  Per-stage and roofline
timings come from a one-stream pass, where kernels do not share the GPU.

Beside it on the same JSON line: the unfiltered 3M-Gaussian dense baseline,
the mask on/off x temporal-cull on/off grid, forward+backward ms/iter
(500k Gaussians, 4 views), mask build time, per-stage event timings with
roofline fractions, and the FP64 CPU oracle timed on a sample of the frame.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/sec at 1352×1014, masked vs dense; fwd+bwd ms/iter @ ≤1e-4 img err"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# fp32 operations the compositor spends on one evaluated (pixel, Gaussian) pair
# on the skip path: offset (2), quadratic form (7), exp2 (1), opacity (1),
# clamp (1), alpha test (1), transmittance test (3).
FLOPS_PER_PAIR = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


# instances per tile above which the range kernel binary-searches each tile's
# two bounds instead of scanning key boundaries (the library's threshold)
RANGES_SEARCH_ABOVE = 2048
# fp32 operations of the adjoint compositor per (pixel, Gaussian) pair it
# differentiates (exponent, alpha, transmittance recovery, colour and alpha
# adjoints, the five geometry terms)
BWD_FLOPS_PER_PAIR = 40
# LDS bytes a wavefront reads per staged record it walks: two 16-byte and one
# 4-byte broadcast read per lane
LDS_BYTES_PER_RECORD_WAVE = 64 * 36


def stage_bytes(name, prof, frames, masked, pixels, n_tiles=None):
    """Algorithmic HBM bytes a stage must move over the profiled frames."""
    P, V, M = prof["processed"], prof["visible"], prof["instances"]
    if name == "preprocess":
        return P * (68 + (4 if masked else 0) + 4) + V * (192 + 64)
    if name == "compact":
        return P * (1 + 4) + V * 8
    if name == "depth_sort":
        return V * 16 * 4
    if name == "offsets":
        return V * (4 + 4 + 8)
    if name == "duplicate":
        return V * 16 + M * 8
    if name == "tile_sort":
        return M * 16 * 2
    if name == "ranges":
        if n_tiles and M / frames > RANGES_SEARCH_ABOVE * n_tiles:
            # two binary searches per tile (one 4-byte key per probe), two bounds written
            probes = 2 * math.ceil(math.log2(max(M / frames, 2)))
            return frames * n_tiles * (probes * 4 + 8)
        return M * 4 + frames * (n_tiles or 0) * 8
    if name == "composite":
        return M * 40 + frames * pixels * 12
    return 0


def source_sha(paths):
    """sha256 (16 hex digits) of the concatenated files."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, name=None):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current sources of that kernel (and, given its full
    name, on the same instantiation).  The file holds one entry or a list of
    entries (one per measured instantiation)."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        data = json.load(f)
    for d in (data if isinstance(data, list) else [data]):
        if name is not None and d.get("kernel") != name:
            continue
        srcs = [os.path.join(ROOT, "paper_2503_16422_amd", "csrc", x) for x in d.get("sources", [])]
        if not srcs or not all(os.path.exists(x) for x in srcs) or source_sha(srcs) != d.get("source_sha"):
            continue
        return d.get("bytes_per_launch")
    return None


def build_masks(ctx, model, cams, n_frames=300, interval=10, mode=1):
    from paper_2503_16422_amd import inputs
    frames = inputs.frame_times(n_frames)
    keys, windows, frame_window = inputs.keyframe_windows(n_frames, interval)
    masks = []
    sync()
    t0 = time.perf_counter()
    for lo, hi in windows:
        bits, idx, count = ctx.build_active_mask(model, frames[lo:hi + 1], frames[lo], frames[hi], mode, cams)
        masks.append((idx, count))
    sync()
    ms = (time.perf_counter() - t0) * 1e3 / len(windows)
    kept = [int(c.item()) for _, c in masks]
    return masks, frame_window, frames, ms, kept


def frame_schedule(k, n_cams, n_frames):
    return k % n_cams, (k * 37 + 11) % n_frames


def run_frames(ctx, model, cams, frames, masks, frame_window, cfg, steps, start, out):
    for k in range(start, start + steps):
        c, f = frame_schedule(k, len(cams), len(frames))
        if masks is None:
            ctx.render(model, cams[c], float(frames[f]), cfg, out_rgb=out)
        else:
            idx, cnt = masks[frame_window[f]]
            ctx.render(model, cams[c], float(frames[f]), cfg, idx=idx, n_idx=cnt, out_rgb=out)


def max_instances(ctx, model, cams, frames, masks, frame_window, cfg, steps, start):
    """Exact instance counts of the frames a timed loop will render."""
    from paper_2503_16422_amd import _lib
    worst = 0
    for k in range(start, start + steps):
        c, f = frame_schedule(k, len(cams), len(frames))
        kw = {}
        if masks is not None:
            idx, cnt = masks[frame_window[f]]
            kw = dict(idx=idx, n_idx=cnt)
        _, _, st = ctx.render(model, cams[c], float(frames[f]), cfg, keep_state=True, **kw)
        worst = max(worst, ctx.binning(st)["n_inst"])
        ctx.release(st)
    return worst


def timed_fps(ctx, model, cams, frames, masks, frame_window, cfg, steps, warmup, out, start=0, prime=False):
    """Frames per second of `steps` frames after `warmup` others.  prime also
    renders the timed frames once beforehand, so that buffers sized by the
    frames' instance counts have grown before the clock starts (the short
    dense loops, whose frames are not sized up front)."""
    run_frames(ctx, model, cams, frames, masks, frame_window, cfg, warmup, start, out)
    if prime:
        run_frames(ctx, model, cams, frames, masks, frame_window, cfg, steps, start + warmup, out)
    sync()
    t0 = time.perf_counter()
    run_frames(ctx, model, cams, frames, masks, frame_window, cfg, steps, start + warmup, out)
    sync()
    dt = time.perf_counter() - t0
    ctx.check_overflow()
    return steps / dt, dt


def timed_fps_pipelined(ctxs, outs, model, cams, frames, masks, frame_window, cfg, steps, warmup, start=0):
    """Frames k = start, start + 1, ... dealt round-robin to len(ctxs) contexts,
    each rendering on a stream of its own into its own image, so that one
    frame's short, low-occupancy launches (preprocess, scans, sorts) run
    beside another frame's compositor.  Every frame is rendered whole; the
    timed region is bracketed by device-wide synchronisations."""
    import torch
    from paper_2503_16422_amd.render import _own_stream
    streams = [_own_stream(c) for c in ctxs]           # one per context, reused (default priority)

    def run(k0, n):
        for k in range(k0, k0 + n):
            j = k % len(ctxs)
            c, f = frame_schedule(k, len(cams), len(frames))
            idx, cnt = masks[frame_window[f]]
            with torch.cuda.stream(streams[j]):
                ctxs[j].render(model, cams[c], float(frames[f]), cfg, idx=idx, n_idx=cnt, out_rgb=outs[j])

    sync()
    run(start, warmup)
    sync()
    t0 = time.perf_counter()
    run(start + warmup, steps)
    sync()
    dt = time.perf_counter() - t0
    for c in ctxs:
        c.check_overflow()
    return steps / dt, dt


def profile_stages(ctx, model, cams, frames, masks, frame_window, cfg, steps, start, out, masked, pixels, n_tiles):
    """Per-stage HIP-event times of `steps` frames (the kernels the timed loop
    runs) and the algorithmic HBM rate of each stage."""
    from paper_2503_16422_amd import _lib
    ctx.profile(True)
    run_frames(ctx, model, cams, frames, masks, frame_window, cfg, steps, start, out)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    stages = {}
    for name in _lib.STAGES[:8]:
        calls = prof["calls"][name]
        if not calls:
            continue
        avg_ms = prof["ms"][name] / calls
        nbytes = stage_bytes(name, prof, steps, masked, pixels, n_tiles)
        entry = {"avg_ms": round(avg_ms, 5), "algorithmic_GBps": round(nbytes / calls / (avg_ms * 1e-3) / 1e9, 1)}
        entry["hbm_frac"] = round(entry["algorithmic_GBps"] / HBM_PEAK_GBS, 4)
        stages[name] = entry
    per_frame = {"processed": prof["processed"] / steps, "visible": prof["visible"] / steps,
                 "instances": prof["instances"] / steps}
    return stages, per_frame


def frame_time_percentiles(ctx, model, cams, frames, masks, frame_window, cfg, steps, start, out):
    """p50 / p99 of per-frame GPU time (HIP events around each frame's
    launches, one stream) over `steps` frames of the loop."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        run_frames(ctx, model, cams, frames, masks, frame_window, cfg, 1, start + k, out)
        ev[k][1].record()
    sync()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return {"p50_ms": round(float(np.percentile(ms, 50)), 4), "p99_ms": round(float(np.percentile(ms, 99)), 4),
            "mean_ms": round(float(ms.mean()), 4), "frames": steps}


def hbm_copy_peak():
    """Device-to-device copy of a 1 GiB buffer: bytes read + written per second."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    sync()
    gbps = 5 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def tiles_of(cfg, W, H):
    return ((W + cfg.tile_w - 1) // cfg.tile_w) * ((H + cfg.tile_h - 1) // cfg.tile_h)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(scene, jobs):
    """FP64 oracle (C, OpenMP, rect mode) rendering whole masked frames.
    jobs: list of (processed indices, camera, t)."""
    import numpy as np
    from oracle import composite as oc
    f32 = lambda x: float(np.float32(x))
    st = oc.Settings(alpha_min=f32(1 / 255), alpha_max=f32(0.99), t_min=f32(1e-4), dilation=f32(0.3))
    t0 = time.perf_counter()
    for idx, cam, t in jobs:
        pre = oc.prepare(scene.arrays(), cam, t, st, idx=idx)
        oc.composite(pre, cam, st, mode="rect")
    dt = time.perf_counter() - t0
    return {"value": len(jobs) / dt, "unit": "frames/s", "cores": oc.num_threads(), "kind": "oracle",
            "sample": f"{len(jobs)} whole masked 1352x1014 frames of the headline workload "
                      f"(~{int(np.mean([j[0].size for j in jobs]))} Gaussians each): FP64 slice, projection and SH "
                      f"in NumPy, then rect-mode per-pixel blending in C/OpenMP; {dt:.1f} s wall",
            "cpu": cpu_model()}


def keyframe_visibility(ctx, model, cams, frames, frame_window, cfg, kept_mode1, out, steps, warmup):
    """The paper's own keyframe masks (Sec. 4.2.2: Gaussians some pixel of some
    view blends at the window's keyframes) and the redundancy measures of
    Sec. 4.1: active ratio |A_t| / N and activation IoU of A_0 and A_t, with
    A_t the Gaussians blended at time t in any of the cameras."""
    import numpy as np
    from paper_2503_16422_amd import _lib
    n = model.n
    a0 = ctx.build_active_mask(model, [], float(frames[0]), float(frames[0]), _lib.MASK_CONTRIBUTED, cams)[0]
    ratio, iou = {}, {}
    for f in range(0, len(frames), 20):
        t = float(frames[f])
        at = ctx.build_active_mask(model, [], t, t, _lib.MASK_CONTRIBUTED, cams)[0]
        ca, cb, cab = (int(x) for x in ctx.mask_overlap(a0, at, n).cpu())
        ratio[f] = round(cb / n, 4)
        iou[f] = round(cab / max(ca + cb - cab, 1), 4)
    masks2, _, _, ms2, kept2 = build_masks(ctx, model, cams, mode=_lib.MASK_CONTRIBUTED)
    worst = max_instances(ctx, model, cams, frames, masks2, frame_window, cfg, steps + warmup, 0)
    cfg2 = _lib.default_cfg(**{k: getattr(cfg, k) for k in ("tile_w", "tile_h", "batch", "pixels_per_thread",
                                                            "schedule")})
    cfg2.instance_capacity = int(worst * 1.05) + 4096
    fps2, _ = timed_fps(ctx, model, cams, frames, masks2, frame_window, cfg2, steps, warmup, out)
    return {"active_ratio_by_frame": ratio, "activation_iou_vs_frame0": iou,
            "contributed_mask_build_ms_per_window": round(ms2, 3),
            "contributed_kept_per_window_mean": int(np.mean(kept2)),
            "kept_vs_tile_mask": round(float(np.mean(kept2)) / float(np.mean(kept_mode1)), 4),
            "masked_fps_contributed_masks_one_stream": round(fps2, 1)}


def finetune_timing(ctx, scene, cams, frames, masks, frame_window, cfg, steps=40):
    """Masked fine-tuning (Sec. 4.2.2) on the headline scene: one 1352x1014 view
    per step, the frame's window mask, every parameter tensor updated by Adam;
    targets rendered from a second scene.  ms per step, host-synchronised
    (the loop reads each step's loss)."""
    from paper_2503_16422_amd import inputs
    from paper_2503_16422_amd.finetune import MaskedFineTuner
    from paper_2503_16422_amd.render import GaussianModel
    model = GaussianModel.from_scene(scene, "cuda:0")
    other = GaussianModel.from_scene(inputs.long_scene(scene.n, seed=1), "cuda:0")
    views, mask_at = [], {}
    for k in range(20):
        c, f = frame_schedule(k * 7, len(cams), len(frames))
        t = float(frames[f])
        mask_at[t] = masks[frame_window[f]]
        idx, cnt = mask_at[t]
        views.append((cams[c], t, ctx.render(other, cams[c], t, cfg, idx=idx, n_idx=cnt)[0].clone()))
    del other
    tuner = MaskedFineTuner(ctx, model, views, mask_of=lambda t: mask_at[t], cfg=cfg)
    for k in range(5):
        tuner.step(k)
    sync()
    t0 = time.perf_counter()
    losses = [tuner.step(k) for k in range(steps)]
    sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_iter": round(ms, 3), "steps": steps, "views": len(views),
            "loss_first_last": [round(losses[0], 1), round(losses[-1], 1)]}


# tile shapes and LDS batches tried for the fwd+bwd loop (the forward autotuner
# times forwards only; here the adjoint decides as much)
# tile shape, LDS batch and pixels per thread (the adjoint takes the forward's 2 or 4)
FWD_BWD_TILES = ((16, 16, 128, 2), (16, 16, 256, 2), (32, 16, 256, 2), (32, 32, 256, 2), (32, 32, 512, 2),
                 (16, 16, 256, 4), (32, 16, 256, 4), (32, 32, 256, 4))


def fwd_bwd(ctx, steps, warmup, streams=3):
    import numpy as np
    import torch
    from paper_2503_16422_amd import _lib, inputs
    from paper_2503_16422_amd.render import Context, GaussianModel, forward_backward_views
    sc = inputs.dense_scene(500_000, seed=0)
    tgt = inputs.dense_scene(500_000, seed=1)
    cams = inputs.arc_cameras(20, 4.0, 1352, 1014)
    rng = np.random.default_rng(2)
    views = [(int(c), float(t)) for c, t in zip(rng.choice(20, 4, replace=False), rng.uniform(0, 1, 4))]
    model = GaussianModel.from_scene(sc, "cuda:0")
    tmodel = GaussianModel.from_scene(tgt, "cuda:0")
    targets = [ctx.render(tmodel, cams[c], t, _lib.default_cfg())[0].clone() for c, t in views]
    grads = {k: torch.zeros_like(getattr(model, k)) for k in GaussianModel.FIELDS}
    states = [None] * 4

    def step(cfg):
        for g in grads.values():
            g.zero_()
        for v, (c, t) in enumerate(views):
            rgb, _, states[v] = ctx.render(model, cams[c], t, cfg, keep_state=states[v] or True)
            dL = rgb - targets[v]
            ctx.backward(states[v], dL, model, grads)

    def release():
        for v, st in enumerate(states):
            if st is not None:
                ctx.release(st)
            states[v] = None

    def timed(cfg, n, nw):
        for _ in range(nw):
            step(cfg)
        sync()
        t0 = time.perf_counter()
        for _ in range(n):
            step(cfg)
        sync()
        return (time.perf_counter() - t0) * 1e3 / n

    sweep = {}
    cfgs = {}
    for tw, th, b, p in FWD_BWD_TILES:
        key = f"{tw}x{th}/b{b}/p{p}"
        cfgs[key] = _lib.default_cfg(tile_w=tw, tile_h=th, batch=b, pixels_per_thread=p, schedule=1)
        sweep[key] = round(timed(cfgs[key], 4, 2), 3)
        release()
    best = min(sweep, key=sweep.get)
    cfg = cfgs[best]
    ms_one = timed(cfg, steps, warmup)
    # the same iteration with consecutive views dealt round-robin to `streams`
    # contexts (one stream each): a view's forward runs beside the previous
    # view's adjoint; the adjoints stay in view order (identical gradients)
    ms = ms_one
    best_p, psweep = best, {}
    if streams > 1:
        # contexts of their own, created together, so that their streams are too
        ctxs = [Context(0) for _ in range(streams)]
        pviews = [(cams[c], t, None, None) for c, t in views]
        pstates = [None] * len(views)

        def ptimed(cfg_p, n, nw):
            nonlocal pstates

            def pstep():
                nonlocal pstates
                for g in grads.values():
                    g.zero_()
                pstates = forward_backward_views(ctxs, model, pviews, cfg_p, lambda v, rgb: rgb - targets[v],
                                                 grads, pstates)

            for _ in range(nw):
                pstep()
            sync()
            t0 = time.perf_counter()
            for _ in range(n):
                pstep()
            sync()
            out_ms = (time.perf_counter() - t0) * 1e3 / n
            for st in pstates:
                st.release()
            pstates = [None] * len(views)
            return out_ms

        # every configuration again with the views in flight, which takes the
        # fastest there
        for key in sweep:
            psweep[key] = round(ptimed(cfgs[key], 10, 3), 3)
        best_p = min(psweep, key=psweep.get)
        ms = ptimed(cfgs[best_p], steps, warmup)
        for c in ctxs:
            c.close()
    cfg = cfgs[best_p]
    ctx.profile(True, count_pairs=True)
    for _ in range(3):
        step(cfg)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    stage_ms = {k: round(v / 3, 4) for k, v in prof["ms"].items() if v > 0}
    release()
    # the adjoint walks the pairs the forward evaluated, back to front
    pairs = prof["pairs"] / 3
    bwd_ms = prof["ms"]["bwd_composite"] / 3
    adj = {"pairs_per_iter": int(pairs), "ms_per_iter": round(bwd_ms, 4),
           "flops_per_pair": BWD_FLOPS_PER_PAIR,
           "achieved_TFLOPs": round(pairs * BWD_FLOPS_PER_PAIR / (bwd_ms * 1e-3) / 1e12, 3)}
    adj["frac_of_fp32_peak"] = round(adj["achieved_TFLOPs"] / FP32_PEAK_TFLOPS, 4)
    return ms, views, stage_ms, {"chosen": best_p, "chosen_one_stream": best, "sweep_ms_per_iter": sweep,
                                 "pipelined_sweep_ms_per_iter": psweep, "one_stream_ms_per_iter": round(ms_one, 3),
                                 "streams": streams}, adj


def batched(ctx, steps=3):
    """8 scenes of uneven size x 64 timestamps x 4 cameras at 800x800, masked,
    rendered by one HIP-graph launch; the tile/batch configuration comes from
    the autotuner run on a 64-view subset."""
    import numpy as np
    import torch
    from paper_2503_16422_amd import _lib, inputs
    from paper_2503_16422_amd.render import GaussianModel
    sizes = inputs.batched_scene_sizes()
    cams = inputs.batch_cameras(800, 800)
    frames = inputs.frame_times(64)
    keys = [0, 13, 26, 39, 52, 63]
    models, masks = [], {}
    sync()
    t0 = time.perf_counter()
    for s, n in enumerate(sizes):
        m = GaussianModel.from_scene(inputs.long_scene(n, seed=s), "cuda:0")
        models.append(m)
        for w in range(len(keys) - 1):
            lo, hi = keys[w], keys[w + 1]
            _, idx, cnt = ctx.build_active_mask(m, frames[lo:hi + 1], frames[lo], frames[hi],
                                                _lib.MASK_TEMPORAL_AND_TILE, cams)
            masks[(s, w)] = (idx, int(cnt.item()))
    sync()
    setup_s = time.perf_counter() - t0
    win = lambda f: min(np.searchsorted(keys, f, side="right") - 1, len(keys) - 2)
    views = []
    for f in range(64):
        for c in range(4):
            for s in range(len(sizes)):
                idx, n = masks[(s, win(f))]
                views.append((s, cams[c], float(frames[f]), idx, n))
    per = 128
    best, sweep = ctx.autotune(models, views[:64], _lib.default_cfg(), views_per_launch=64, repeats=2)
    cfg = _lib.default_cfg(tile_w=best.tile_w, tile_h=best.tile_h, batch=best.batch,
                           pixels_per_thread=best.pixels_per_thread, schedule=best.schedule)
    out = torch.empty((len(views), 3, 800, 800), dtype=torch.float32, device="cuda")
    ctx.profile(True)
    ctx.render_batch(models, views, cfg, views_per_launch=per, out=out)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    n_launch = (len(views) + per - 1) // per
    cap = int(prof["instances"] / n_launch * 1.5) + 65536
    for _ in range(3):
        cfg.instance_capacity = cap
        ctx.render_batch(models, views, cfg, views_per_launch=per, use_graph=True, out=out)
        try:
            ctx.check_overflow()
            break
        except _lib.FdgsError:
            cap *= 2
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.render_batch(models, views, cfg, views_per_launch=per, use_graph=True, out=out)
    sync()
    dt = (time.perf_counter() - t0) / steps
    ctx.check_overflow()
    return {"views": len(views), "resolution": [800, 800], "scenes": sizes, "views_per_launch": per,
            "graph_ms_per_batch": round(dt * 1e3, 2), "views_per_s": round(len(views) / dt, 1),
            "instances_per_view": int(prof["instances"] / len(views)),
            "autotuned": {"tile": [best.tile_w, best.tile_h], "batch": best.batch,
                          "pixels_per_thread": best.pixels_per_thread, "schedule": best.schedule},
            "autotune_sweep_ms_64_views": {f"{r['tile'][0]}x{r['tile'][1]}/b{r['batch']}/p{r['pixels_per_thread']}/s{r['schedule']}":
                                           round(r["ms"], 3) for r in sweep},
            "setup_s": round(setup_s, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--streams", type=int, default=4,
                    help="headline frames dealt round-robin over this many streams (one context each)")
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="hardware queues HIP gives this process (GPU_MAX_HW_QUEUES, set before HIP starts; "
                         "HIP's default is 4, of which the default stream, which builds the masks and runs "
                         "the one-stream pass, holds one: more frame streams than three then share queues); "
                         "0 leaves the environment as it is")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the masked headline loop (for profiler runs)")
    ap.add_argument("--config", default=None,
                    help="tile_w,tile_h,batch,pixels_per_thread,schedule: skip the autotuner and use this "
                         "configuration")
    ap.add_argument("--dense-vanilla-only", action="store_true",
                    help="only a few dense 3M-Gaussian unfiltered frames (for profiler runs)")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="only the forward+backward loop (500k Gaussians, 4 views; for profiler runs)")
    ap.add_argument("--fwd-bwd-streams", type=int, default=3,
                    help="contexts (one stream each) the fwd+bwd iteration deals its views to")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 256 MiB buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build renders every view on a single MI355X and has no "
              "multi-GPU path (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)
    if args.streams < 1:
        print("--streams must be at least 1", file=sys.stderr)
        sys.exit(2)
    if not 0 <= args.hw_queues <= 32:
        print("--hw-queues must be in [0, 32]", file=sys.stderr)
        sys.exit(2)
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)   # before the HIP runtime starts (torch import)

    import numpy as np
    import torch
    from paper_2503_16422_amd import _lib, inputs
    from paper_2503_16422_amd.render import Context, GaussianModel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = Context(0)
    # measured rates of this device: HBM by a 1 GiB copy, LDS and VALU by micro-benchmarks
    peaks = ctx.measure_peaks()
    peaks["hbm_copy_GBps"] = round(hbm_copy_peak(), 1)
    log(f"[bench] measured peaks: {json.dumps(peaks)}")
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        sync()
        del a, b
    if args.fwd_bwd_only:
        ms_iter, views, fb_stages, fb_tiles, _ = fwd_bwd(ctx, args.steps, args.warmup, args.fwd_bwd_streams)
        log(f"[bench] fwd+bwd {ms_iter:.2f} ms/iter; tiles {fb_tiles}; stages {json.dumps(fb_stages)}")
        return
    W, H = 1352, 1014
    cams = inputs.arc_cameras(20, 4.0, W, H)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    if args.dense_vanilla_only:
        dmodel = GaussianModel.from_scene(inputs.dense_scene(3_000_000, seed=0), "cuda:0")
        frames = inputs.frame_times(300)
        vanilla = _lib.default_cfg(temporal_cull=0, tile_cull=0)
        d_fps, _ = timed_fps(ctx, dmodel, cams, frames, None, None, vanilla, args.steps, args.warmup, out,
                             start=2000, prime=True)
        log(f"[bench] dense vanilla {d_fps:.1f} frames/s")
        return

    # ---- headline: masked 200k scene -------------------------------------------------
    log("[bench] masked scene: generating 200k Gaussians")
    scene = inputs.long_scene(200_000, seed=0)
    model = GaussianModel.from_scene(scene, "cuda:0")
    masks, frame_window, frames, mask_ms, kept = build_masks(ctx, model, cams)
    log(f"[bench] masks: {len(masks)} windows, {mask_ms:.2f} ms/window, kept mean {np.mean(kept):.0f}")
    K, Wu = args.steps, args.warmup
    # autotune tile shape / LDS batch / pixels per thread on 24 frames of the workload
    tune_views = []
    for k in range(24):
        c, f = frame_schedule(k * 13, len(cams), len(frames))
        idx, cnt = masks[frame_window[f]]
        tune_views.append((0, cams[c], float(frames[f]), idx, int(cnt.item())))
    refine, refine_pipe = {}, {}
    # the contexts (one stream and image each) that frames are dealt to
    ctxs = [ctx] + [Context(0) for _ in range(args.streams - 1)]
    outs = [out] + [torch.empty_like(out) for _ in range(args.streams - 1)]
    if args.config:
        tw, th, b, p, sc = (int(x) for x in args.config.split(","))
        tuned, sweep = dict(tile_w=tw, tile_h=th, batch=b, pixels_per_thread=p, schedule=sc), []
        tuned1 = tuned
    else:
        best, sweep = ctx.autotune([model], tune_views, _lib.default_cfg(), views_per_launch=1, repeats=2)
        tuned = dict(tile_w=best.tile_w, tile_h=best.tile_h, batch=best.batch,
                     pixels_per_thread=best.pixels_per_thread, schedule=best.schedule)
        # the sweep's six fastest, timed again the way the benchmark loops run
        # (fixed capacity, 200 frames; on one stream, and dealt over the
        # streams), so that near-ties are settled on the loops themselves: the
        # one-stream rate and the pipelined rate each take their own fastest
        # (with frames in flight a smaller LDS batch can win by leaving room on
        # a CU for the other frames' short launches)
        # each candidate is timed twice, in two interleaved passes over the
        # candidates, and keeps its better rate (single runs differ by a few
        # percent from one to the next)
        tuned1 = tuned
        cands = []
        for r in sorted(sweep, key=lambda r: r["ms"])[:6]:
            cand = dict(tile_w=r["tile"][0], tile_h=r["tile"][1], batch=r["batch"],
                        pixels_per_thread=r["pixels_per_thread"], schedule=r["schedule"])
            n_inst = max_instances(ctx, model, cams, frames, masks, frame_window, _lib.default_cfg(**cand), 210, 0)
            cands.append((cand, _lib.default_cfg(instance_capacity=int(n_inst * 1.05) + 4096, **cand)))
        for _ in range(2):
            for cand, cfg_c in cands:
                key = tuple(cand.values())
                f_c, _ = timed_fps(ctx, model, cams, frames, masks, frame_window, cfg_c, 200, 10, out)
                refine[key] = max(refine.get(key, 0.0), f_c)
                if args.streams > 1:
                    f_p, _ = timed_fps_pipelined(ctxs, outs, model, cams, frames, masks, frame_window, cfg_c, 200,
                                                 10)
                    refine_pipe[key] = max(refine_pipe.get(key, 0.0), f_p)
        tuned1 = dict(zip(cands[0][0].keys(), max(refine, key=refine.get)))
        tuned = dict(zip(cands[0][0].keys(), max(refine_pipe, key=refine_pipe.get))) if refine_pipe else tuned1
        log(f"[bench] autotune refinement (frames/s, best of two 200-frame runs, one stream): "
            f"{ {'/'.join(str(x) for x in k): round(v, 1) for k, v in refine.items()} }")
        if refine_pipe:
            log(f"[bench] autotune refinement (frames/s, best of two 200-frame runs, {args.streams} streams): "
                f"{ {'/'.join(str(x) for x in k): round(v, 1) for k, v in refine_pipe.items()} }")
    log(f"[bench] autotuned {tuned} (one stream: {tuned1})")
    worst = max_instances(ctx, model, cams, frames, masks, frame_window, _lib.default_cfg(**tuned), K + Wu, 0)
    worst1 = worst if tuned1 == tuned else max_instances(ctx, model, cams, frames, masks, frame_window,
                                                         _lib.default_cfg(**tuned1), K + Wu, 0)
    log(f"[bench] max instances over the timed frames {worst}")
    cap = int(worst * 1.05) + 4096
    cfg_default = _lib.default_cfg(instance_capacity=int(
        max_instances(ctx, model, cams, frames, masks, frame_window, _lib.default_cfg(), K + Wu, 0) * 1.05) + 4096)
    fps_default, _ = timed_fps(ctx, model, cams, frames, masks, frame_window, cfg_default, K, Wu, out)
    # cfg: the configuration the headline value is timed in (and its stages,
    # roofline and counters); cfg1: the one-stream rate's own
    cfg = _lib.default_cfg(instance_capacity=cap, **tuned)
    cfg1 = _lib.default_cfg(instance_capacity=int(worst1 * 1.05) + 4096, **tuned1)
    fps1, dt = timed_fps(ctx, model, cams, frames, masks, frame_window, cfg1, K, Wu, out)
    log(f"[bench] masked, one stream: {fps1:.1f} frames/s ({dt * 1e3 / K:.3f} ms/frame); default config "
        f"{fps_default:.1f}")
    fps = fps1
    if args.streams > 1:
        fps, dt = timed_fps_pipelined(ctxs, outs, model, cams, frames, masks, frame_window, cfg, K, Wu)
        log(f"[bench] masked, frames pipelined over {args.streams} streams: {fps:.1f} frames/s")
    for c in ctxs[1:]:
        c.close()
    del outs, ctxs

    # same frames again with stage events (the kernels that ran timed), then
    # once more with the compositor's pair-counting variant for the pair count
    ctx.profile(True)
    run_frames(ctx, model, cams, frames, masks, frame_window, cfg, K, Wu, out)
    prof = ctx.profile_read(reset=True)
    ctx.profile(True, count_pairs=True)
    run_frames(ctx, model, cams, frames, masks, frame_window, cfg, K, Wu, out)
    pp = ctx.profile_read(reset=True)
    prof["pairs"], prof["blended"] = pp["pairs"], pp["blended"]
    ctx.profile(False)
    stages = {}
    for name in _lib.STAGES[:8]:
        calls = prof["calls"][name]
        if not calls:
            continue
        avg_ms = prof["ms"][name] / calls
        nbytes = stage_bytes(name, prof, K, True, W * H, tiles_of(cfg, W, H))
        entry = {"avg_ms": round(avg_ms, 5), "algorithmic_GBps": round(nbytes / calls / (avg_ms * 1e-3) / 1e9, 1)}
        entry["hbm_frac"] = round(entry["algorithmic_GBps"] / HBM_PEAK_GBS, 4)
        entry["hbm_frac_of_copy"] = round(entry["algorithmic_GBps"] / peaks["hbm_copy_GBps"], 4)
        stages[name] = entry
    comp = stages["composite"]
    pairs_per_frame = prof["pairs"] / K
    comp_tflops = pairs_per_frame * FLOPS_PER_PAIR / (comp["avg_ms"] * 1e-3) / 1e12
    comp["pairs_per_frame"] = int(pairs_per_frame)
    # pairs that blended (alpha >= alpha_min while the pixel is live): the rest
    # are evaluated because the pixel's wavefront cell is reached by the ellipse
    comp["blended_pairs_per_frame"] = int(prof["blended"] / K)
    comp["blended_fraction"] = round(prof["blended"] / max(prof["pairs"], 1), 4)
    comp["achieved_TFLOPs"] = round(comp_tflops, 3)
    comp["valu_frac_of_measured"] = round(pairs_per_frame * FLOPS_PER_PAIR / 2 / (comp["avg_ms"] * 1e-3)
                                          / peaks["valu_fma_lane_ops_per_s"], 4)
    # LDS: every (record, wavefront) the walk visits reads the staged record;
    # a wavefront evaluates 64 x pixels-per-thread pairs per record it walks
    lds_bps = pairs_per_frame / (64 * cfg.pixels_per_thread) * LDS_BYTES_PER_RECORD_WAVE / (comp["avg_ms"] * 1e-3)
    comp["lds_TBps"] = round(lds_bps / 1e12, 2)
    comp["lds_frac_of_measured"] = round(lds_bps / peaks["lds_broadcast_Bps"], 4)
    # the paper's two rates: "FPS" times the whole render call (host work
    # included: fps1), "Raster FPS" the rasterisation alone (GPU time of a
    # frame's launches, events around each frame)
    frame_pct = frame_time_percentiles(ctx, model, cams, frames, masks, frame_window, cfg1, K, Wu, out)
    raster_ms = frame_pct["mean_ms"]
    log(f"[bench] frame time {frame_pct}")
    dominant = max(stages, key=lambda s: stages[s]["avg_ms"])
    if dominant == "composite":
        kname = (f"composite_kernel<{cfg.tile_w}, {cfg.tile_h}, {cfg.batch}, {cfg.pixels_per_thread}, 0, "
                 f"{'true' if cfg.schedule else 'false'}>")
        roof = {"bound": "alu", "kernel": kname, "achieved": round(comp_tflops, 3),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(comp_tflops / FP32_PEAK_TFLOPS, 4),
                "traffic": load_traffic("composite", kname)}
    else:
        e = stages[dominant]
        roof = {"bound": "hbm", "kernel": dominant, "achieved": e["algorithmic_GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": e["hbm_frac"], "traffic": load_traffic(dominant)}
    per_frame = {"processed": prof["processed"] / K, "visible": prof["visible"] / K,
                 "instances": prof["instances"] / K}
    log(f"[bench] stages: {json.dumps(stages)}")

    extra = {}
    if not args.headline_only:
        # ---- forward + backward ------------------------------------------------------
        log("[bench] fwd+bwd: 500k Gaussians, 4 views")
        ms_iter, views, fb_stages, fb_tiles, adj = fwd_bwd(ctx, 50, 5, args.fwd_bwd_streams)
        extra["fwd_bwd_ms_per_iter"] = round(ms_iter, 3)
        extra["fwd_bwd_stage_ms_per_iter"] = fb_stages
        extra["fwd_bwd_adjoint_compositor"] = adj
        extra["fwd_bwd_config"] = {"gaussians": 500_000, "views": views, "resolution": [W, H],
                                   "loss": "0.5*sum((I-I*)^2), targets rendered from a second seed",
                                   "tiles": fb_tiles}
        log(f"[bench] fwd+bwd {ms_iter:.2f} ms/iter ({fb_tiles})")

        # ---- mask on/off x temporal cull on/off on the same scene ---------------------
        grid = {}
        n_grid = 60
        for use_mask in (True, False):
            for cull in (1, 0):
                c0 = _lib.default_cfg(temporal_cull=cull)
                f, _ = timed_fps(ctx, model, cams, frames, masks if use_mask else None, frame_window, c0,
                                 n_grid, 5, out, start=1000)
                grid[f"mask={'on' if use_mask else 'off'},cull={'on' if cull else 'off'}"] = round(f, 1)
        for use_mask in (True, False):
            c0 = _lib.default_cfg(temporal_cull=int(use_mask), tile_cull=0)
            f, _ = timed_fps(ctx, model, cams, frames, masks if use_mask else None, frame_window, c0,
                             n_grid, 5, out, start=1000)
            key = "mask=on,cull=on" if use_mask else "mask=off,cull=off"
            grid[key + ",tile_cull=off"] = round(f, 1)
        log(f"[bench] grid: {grid}")
        extra["masked_scene_grid_fps"] = grid

        # ---- the paper's keyframe visibility masks, active ratio and IoU ---------------
        extra["keyframe_visibility"] = keyframe_visibility(ctx, model, cams, frames, frame_window, cfg1, kept, out,
                                                           K, Wu)
        log(f"[bench] keyframe visibility: {json.dumps(extra['keyframe_visibility'])}")

        # ---- masked fine-tuning step time ------------------------------------------
        ft_cfg = _lib.default_cfg(instance_capacity=0)
        extra["masked_finetune"] = finetune_timing(ctx, scene, cams, frames, masks, frame_window, ft_cfg)
        log(f"[bench] masked fine-tuning: {json.dumps(extra['masked_finetune'])}")

        # ---- SH vector quantisation (post-processing): codebook build, then the same frames --
        k_vq, it_vq = 4096, 10
        ctx.sh_kmeans(model, k_vq, 1)                                  # warm-up (allocations)
        sync()
        t0 = time.perf_counter()
        code, assign = ctx.sh_kmeans(model, k_vq, it_vq)
        sync()
        vq_s = time.perf_counter() - t0
        qmodel = model.quantized(assign, code)
        q_fps, _ = timed_fps(ctx, qmodel, cams, frames, masks, frame_window, cfg1, K, Wu, out)
        extra["sh_vq"] = {"codebook": k_vq, "iterations": it_vq, "kmeans_s": round(vq_s, 4),
                          "sh_bytes_dense": int(model.n * 192), "sh_bytes_vq": int(model.n * 4 + k_vq * 192),
                          "masked_fps_vq": round(q_fps, 1)}
        log(f"[bench] sh vq: {json.dumps(extra['sh_vq'])}")
        del qmodel, code, assign

        # ---- dense unfiltered 3M scene -----------------------------------------------
        del model
        torch.cuda.empty_cache()
        log("[bench] dense scene: generating 3M Gaussians")
        dense = inputs.dense_scene(3_000_000, seed=0)
        dmodel = GaussianModel.from_scene(dense, "cuda:0")
        del dense
        n_dense = 16
        vanilla = _lib.default_cfg(temporal_cull=0, tile_cull=0)
        d_fps, _ = timed_fps(ctx, dmodel, cams, frames, None, frame_window, vanilla, n_dense, 3, out, start=2000,
                             prime=True)
        d_stages, d_work = profile_stages(ctx, dmodel, cams, frames, None, frame_window, vanilla, n_dense, 2003,
                                          out, False, W * H, tiles_of(vanilla, W, H))
        d_pct = frame_time_percentiles(ctx, dmodel, cams, frames, None, frame_window, vanilla, n_dense, 2003, out)
        log(f"[bench] dense vanilla stages: {json.dumps(d_stages)}")
        dt_fps, _ = timed_fps(ctx, dmodel, cams, frames, None, frame_window, _lib.default_cfg(temporal_cull=0),
                              n_dense, 3, out, start=2000, prime=True)
        dc_fps, _ = timed_fps(ctx, dmodel, cams, frames, None, frame_window, _lib.default_cfg(), n_dense, 3, out,
                              start=2000, prime=True)
        dmasks, dfw, _, dmask_ms, dkept = build_masks(ctx, dmodel, cams)
        dm_fps, _ = timed_fps(ctx, dmodel, cams, frames, dmasks, dfw, _lib.default_cfg(), 60, 5, out, start=2000)
        log(f"[bench] dense: vanilla {d_fps:.1f}, +tile cull {dt_fps:.1f}, +temporal cull {dc_fps:.1f}, "
            f"+mask {dm_fps:.1f} frames/s")
        extra["dense_3M"] = {"vanilla_fps": round(d_fps, 2), "vanilla_stages": d_stages,
                             "vanilla_frame_time": d_pct,
                             "vanilla_per_frame": {k: int(v) for k, v in d_work.items()},
                             "vanilla_tile_cull_fps": round(dt_fps, 2),
                             "temporal_cull_fps": round(dc_fps, 2),
                             "masked_fps": round(dm_fps, 2), "mask_build_ms_per_window": round(dmask_ms, 2),
                             "kept_mean": int(np.mean(dkept))}
        # like for like: both rates from one stream, one frame after another
        extra["masked_200k_vs_dense_3M_vanilla_one_stream"] = round(fps1 / d_fps, 2)
        del dmodel, dmasks
        torch.cuda.empty_cache()

        # ---- batched multi-view render (HIP graph + autotuner) ------------------------
        log("[bench] batched: 8 scenes x 64 t x 4 cameras at 800x800")
        extra["batched_2048_views"] = batched(ctx)
        log(f"[bench] batched: {json.dumps(extra['batched_2048_views'])}")
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline and not args.headline_only:
        jobs = []
        for k in range(3):
            c, f = frame_schedule(Wu + k, len(cams), len(frames))
            idx, cnt = masks[frame_window[f]]
            sel = idx[: int(cnt.item())].cpu().numpy().view(np.uint32).astype(np.int64)
            jobs.append((sel, cams[c], float(frames[f])))
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(scene, jobs)
        log(f"[bench] cpu baseline {cpu['value']:.4f} frames/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": Wu,
        "ms_per_step": round(1e3 / fps, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (per-Gaussian geometry f64)", "data": "synthetic",
        "config": {"workload": "masked 4D Gaussian frame: 200k long-lifespan Gaussians (log s_t~N(-1,0.4)), "
                               "1352x1014, 20 cameras x 300 timestamps, keyframe masks every 10 frames "
                               "(temporal and tile predicate)",
                   "autotuned": tuned, "autotuned_one_stream": tuned1, "streams": args.streams,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")), "one_stream_fps": round(fps1, 2),
                   "default_config_fps": round(fps_default, 2),
                   "autotune_refinement_fps": {"/".join(str(x) for x in k): round(v, 1) for k, v in refine.items()},
                   "autotune_refinement_pipelined_fps": {"/".join(str(x) for x in k): round(v, 1)
                                                         for k, v in refine_pipe.items()},
                   "autotune_sweep_ms_per_frame": {
                       f"{r['tile'][0]}x{r['tile'][1]}/b{r['batch']}/p{r['pixels_per_thread']}/s{r['schedule']}":
                       round(r["ms"] / len(tune_views), 4) for r in sweep},
                   "gaussians": 200_000, "resolution": [W, H], "mask_windows": len(masks),
                   "kept_per_window_mean": int(np.mean(kept)), "per_frame": per_frame,
                   "mask_build_ms_per_window": round(mask_ms, 3),
                   "raster_fps_one_stream": round(1e3 / raster_ms, 1), "frame_time_one_stream": frame_pct},
        "roofline": roof,
        "peaks_measured": peaks,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
