#!/usr/bin/env python
"""Throughput of masked forward + backward rasterization on one MI355X.

A step is one pass of the hot path over one batch of synthetic input:
straight-through Gumbel mask sampling, projection, tile counts, scan, key
duplication, radix sort, tile ranges, masked compositing, L1 loss gradient,
masked backward compositing, projection backward and the mask-score
gradient.  The default workload is the batched multi-view case: a
1M-Gaussian unbounded scene (SH degree 3, heavy-tailed scales) rendered for
8 views of uneven size in one call ("batched"), compared with 8 single-view
calls ("plain").

metric: Gaussian-pixel evaluations per second, counting for every pixel the
sorted entries its 16x16 tile list presents up to and including its stop
entry (the forward evaluations; each has a backward counterpart).

Prints one JSON line.  --gpus N > 1 is rejected: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU lane-slots per Gaussian-pixel evaluation, counted from the formulas
# (each add, multiply, fused multiply-add, compare or select is one slot; exp
# and reciprocal are quarter rate and count four).
SLOTS_FILTER = 16      # dx, dy, Q, cut, exp, o*G, clamp, alpha filter
SLOTS_BLEND = 9        # M*a, test, stop compare, weight, 3 colour FMAs, T
SLOTS_BWD_VISIBLE = 44  # T recovery (rcp), X, dL/dM, dL/dc, dL/do, dL/dQ, dL/du,dv, conic, b update
SLOTS_BWD_MASKED = 11   # X with T unchanged, dL/dM
PEAK_SLOTS = 256 * 64 * 2.4e9   # 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz
PEAK_HBM = 8.0e12


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def build_workload(name: str):
    import scenegen
    if name == "batched":
        s = scenegen.batched_scene()
        desc = "batched: 1M-Gaussian unbounded scene (SH3, heavy-tailed scales), 8 uneven views in one call"
    elif name == "unbounded":
        s = scenegen.unbounded_scene()
        desc = "unbounded: 1.5M Gaussians (SH3, heavy-tailed scales), one 1264x832 view"
    elif name == "object":
        s = scenegen.object_scene()
        desc = "object: 200k Gaussians in 64 clusters (SH3), one 800x800 view"
    elif name == "tiny":
        s = scenegen.tiny_scene()
        desc = "tiny: 4096 Gaussians (SH0), one 128x128 view"
    else:
        raise SystemExit(f"unknown workload {name}")
    return s, desc


def stage_roofline(stage: str, ms_per_launch: float, counts: dict, frame_stats: dict, n: int, views: int,
                   sh_deg: int):
    """Algorithmic work of one launch of `stage` and its roofline."""
    t = ms_per_launch * 1e-3
    K = frame_stats["n_instances"]
    R = frame_stats["n_records"]
    P = frame_stats["n_pixels"]
    k3 = 3 * (sh_deg + 1) ** 2
    if stage == "composite_bwd":
        # entries the backward evaluates: those up to each pixel's last blended
        # one that can reach a pixel of their tile
        vis = counts["blended"] - counts["blended_masked"]
        work = SLOTS_FILTER * counts["bwd_evaluated"] + SLOTS_BWD_VISIBLE * vis + SLOTS_BWD_MASKED * counts[
            "blended_masked"]
        return dict(bound="alu", achieved=work / t / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                    frac=work / t / PEAK_SLOTS, algorithmic=work, algorithmic_unit="VALU lane-slots")
    if stage == "composite_fwd":
        work = SLOTS_FILTER * counts["evaluated"] + SLOTS_BLEND * counts["blended"]
        return dict(bound="alu", achieved=work / t / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                    frac=work / t / PEAK_SLOTS, algorithmic=work, algorithmic_unit="VALU lane-slots")
    if stage == "sort":
        # stable pass over 32-bit tile keys and 32-bit values: read and write both
        passes = frame_stats["sort_passes"]
        byt = 16 * K * passes
    elif stage == "depth_sort":
        byt = 16 * R * 4 + R * 12
    elif stage == "project":
        byt = n * 4 * (11 + k3 + 1) + R * (48 + 12)
    elif stage == "project_bwd":
        byt = n * 4 * (11 + k3) + R * 36 + n * 4 * (10 + k3)
    elif stage == "duplicate":
        byt = R * 16 + K * 12
    elif stage == "scan":
        byt = R * 8
    else:
        byt = P * 16
    return dict(bound="hbm", achieved=byt / t / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s", frac=byt / t / PEAK_HBM,
                algorithmic=byt, algorithmic_unit="bytes")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "counters_batched1M_8views.txt")
TRAFFIC_SOURCES = ("hybrid.hip", "composite_common.hpp", "common.hpp")


def measured_traffic(stage: str):
    """HBM bytes per launch of a compositing kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        line = next(l for l in open(TRAFFIC_FILE) if l.startswith("traffic: "))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line[len("traffic: "):])
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2412_20522_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16") or stage not in rec:
        return None
    return rec[stage]["bytes"]


def cpu_baseline(scene: dict, tau: float, seed: int, step: int, min_seconds: float = 10.0) -> dict:
    """The FP64 oracle on a bounded sample of the same workload: the views
    of the batched step, one at a time (same masks, full masked fwd+bwd
    through the projection backward), until at least `min_seconds` have
    passed."""
    import oracle
    oracle.lib()
    ost = oracle.RasterSettings(sh_degree=scene["sh_degree"])
    m, _ = oracle.sample_masks(scene["mask_scores"], tau, seed, step)
    cams = scene["cameras"]
    evals, done, dt = 0, [], 0.0
    k = 0
    while dt < min_seconds:
        v = k % len(cams)
        cam = cams[v]
        t0 = time.perf_counter()
        out = oracle.run_pipeline(scene, [cam], m, ost, targets=[scene["targets"][v]])
        dt += time.perf_counter() - t0
        evals += int(out.fwd.examined.sum())
        done.append(f"{cam['width']}x{cam['height']}")
        k += 1
    return {"value": evals / dt, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(done)} single-view fwd+bwd passes of the same scene and masks (views {', '.join(done)}), "
                      f"FP64, {evals} evals in {dt:.1f} s",
            "views_per_s": len(done) / dt, "seconds": dt}


def prune_and_render(rast, params: dict, n: int, cams, seed: int, reps: int = 20) -> dict:
    """Probabilistic pruning (10 draws) of a whole per-Gaussian training state
    (parameters, mask scores and both Adam moments of each: 183 floats per
    Gaussian) whose scores are those of late training (62.4 % of the Gaussians
    with scores that all but rule them out, Sec. 4.2), timed with HIP events;
    then forward-only rendering (all masks 1) of the full and of the pruned
    set on a fixed workspace, as views per second."""
    import torch
    import scenegen
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import PARAM_KEYS
    dev = params["means"].device
    scores = torch.from_numpy(scenegen.converged_mask_scores(n)).to(dev)
    state = dict(params)
    for k, v in list(params.items()) + [("scores", scores)]:
        state[f"adam_m_{k}"] = torch.zeros_like(v)
        state[f"adam_v_{k}"] = torch.zeros_like(v)
    names = ["scores", *state.keys()]
    ins = [scores, *state.values()]
    floats = sum(t.numel() for t in ins) // n
    keep = torch.empty(n, dtype=torch.int32, device=dev)
    outs = [torch.empty_like(t) for t in ins]
    n_kept = torch.zeros(1, dtype=torch.int64, device=dev)
    scratch = torch.empty(int(M.lib().mgs_compact_scratch_bytes(n)), dtype=torch.uint8, device=dev)

    def prune_once(step0):
        M.mgs_prune_sample(rast.ctx, scores, seed, step0, 10, keep)
        M.mgs_compact_rows(rast.ctx, keep, ins, outs, n_kept=n_kept, scratch=scratch)

    prune_once(20_000)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        prune_once(20_000 + 10 * r)
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / reps
    k = int(n_kept.item())
    # algorithmic bytes: scores read by the draws, keep written and read twice
    # (scan, compaction), every row read, the kept rows written
    moved = 8 * n + 12 * n + 4 * floats * (n + k)
    pruned = {name: t[:k] for name, t in zip(names, outs)}

    frames = []

    def render_ms(ps: dict, count: int, importance: bool = False) -> float:
        fr = rast.acquire_frame()  # a frame of its own (fixed workspaces are per frame)
        frames.append(fr)
        ones = torch.ones(count, device=dev)
        imgs = torch.empty(3 * sum(c["width"] * c["height"] for c in cams), device=dev)
        isum, imax = torch.empty(count, device=dev), torch.empty(count, device=dev)

        def once():
            if importance:
                rast.forward_importance(fr, ps, ones, cams, images=imgs, imp_sum=isum, imp_max=imax)
            else:
                rast.forward(fr, ps, ones, cams, images=imgs)

        once()
        rast.reserve(fr, 1.25)  # fixed workspace: no host synchronisation per forward
        for _ in range(2):
            once()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            once()
        b.record()
        torch.cuda.synchronize()
        rast.check(fr)
        return a.elapsed_time(b) / reps

    full_ms = render_ms(params, n)
    pr_ms = render_ms({key: pruned[key] for key in PARAM_KEYS}, k)
    imp_ms = render_ms(params, n, importance=True)
    for fr in frames:
        rast.release_frame(fr)
    V = len(cams)
    return {
        "prune": {"ms": pms, "gaussians": n, "kept": k, "draws": 10, "floats_per_gaussian": floats,
                  "scores": "62.4 % of the Gaussians with s0 - s1 = -8, the rest +8 (seeded)",
                  "algorithmic_bytes": moved, "GB_per_s": moved / (pms * 1e-3) / 1e9},
        "render_only": {"full": {"ms": full_ms, "views_per_s": V / (full_ms * 1e-3), "gaussians": n},
                        "pruned": {"ms": pr_ms, "views_per_s": V / (pr_ms * 1e-3), "gaussians": k},
                        "speedup": full_ms / pr_ms},
        "importance": {"ms": imp_ms, "overhead_vs_forward": imp_ms / full_ms - 1.0,
                       "what": "forward-only render of the full set that also returns every Gaussian's sum and "
                               "max of M alpha T"},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched", choices=["batched", "unbounded", "object", "tiny"])
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the pruning and forward-only timings")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--batch-depth", type=int, default=128)
    ap.add_argument("--fwd-ppt", type=int, default=4)
    ap.add_argument("--bwd-ppt", type=int, default=4)
    ap.add_argument("--persistent", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1, help="pick tile shape / batch depth / pixels per thread")
    ap.add_argument("--graph", type=int, default=1, help="time replays of a hipGraph-captured step")
    ap.add_argument("--tile-cull", type=int, default=1, help="narrow instances only for reachable tiles")
    ap.add_argument("--wide-tiles", type=int, default=8,
                    help="hybrid binning threshold in tiles (0: automatic, -1: every record duplicated)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; runs on several GPUs are not supported (got --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import PARAM_KEYS, Grads, Rasterizer

    if args.copy_calibration_mib > 0:
        # a plain copy of known size: reads and writes exactly this many bytes
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {nbytes} bytes")
        del src, dst

    t_gen = time.perf_counter()
    scene, desc = build_workload(args.workload)
    log(f"[bench] generated {scene['name']} in {time.perf_counter() - t_gen:.1f} s")
    cams = scene["cameras"]
    V = len(cams)
    n = scene["means"].shape[0]
    deg = scene["sh_degree"]
    tau = float(scene.get("gumbel_tau", 0.5))
    lambda_m, seed, step_id = 0.1, 2412, 0
    dev = torch.device("cuda:0")
    params = {k: torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).to(dev) for k in PARAM_KEYS}
    scores = torch.from_numpy(scene["mask_scores"]).to(dev)
    P = sum(c["width"] * c["height"] for c in cams)
    targets = torch.cat([torch.from_numpy(t.reshape(-1)) for t in scene["targets"]]).to(dev)
    tw, th = (int(x) for x in args.tile.split("x"))
    rast = Rasterizer(0, sh_degree=deg, tile_w=tw, tile_h=th, batch_depth=args.batch_depth, fwd_ppt=args.fwd_ppt,
                      bwd_ppt=args.bwd_ppt, persistent=args.persistent, wide_tiles=args.wide_tiles,
                      tile_cull=args.tile_cull)
    ctx = rast.ctx
    frame = rast.acquire_frame()
    images = torch.empty(3 * P, device=dev)
    d_img = torch.empty_like(images)
    loss = torch.zeros(1, device=dev)
    loss_m = torch.zeros(1, device=dev)
    grads = Grads(*(torch.empty_like(params[k]) for k in PARAM_KEYS), torch.empty(n, device=dev))
    d_scores = torch.empty(n, 2, device=dev)
    m_hard = torch.empty(n, device=dev)
    y_soft = torch.empty(n, device=dev)
    red_scratch = torch.empty(int(M.lib().mgs_reduce_scratch_bytes(3 * P)), dtype=torch.uint8, device=dev)

    def batched_step():
        M.mgs_sample_masks(ctx, scores, tau, seed, step_id, m_hard, y_soft)
        rast.forward(frame, params, m_hard, cams, images=images)
        M.mgs_l1_loss_grad(ctx, images, targets, d_img, loss, red_scratch)
        rast.backward(frame, params, d_img, out=grads)
        M.mgs_mask_grad(ctx, grads.masks, m_hard, y_soft, tau, lambda_m, d_scores, loss_m, red_scratch)

    # the evaluation count at 16x16 tiles (the numerator), untimed
    # (lists of Sec. 3.1 exactly: no tile culling, so the count is that of the
    # full lists whatever the timed configuration skips)
    rast.set(tile_w=16, tile_h=16, fwd_ppt=1, bwd_ppt=4, persistent=0, tile_cull=0)
    M.mgs_sample_masks(ctx, scores, tau, seed, step_id, m_hard, y_soft)
    rast.forward(frame, params, m_hard, cams, images=images)
    counts16 = rast.count_evals(frame)
    E16 = counts16["examined"]
    rast.set(tile_w=tw, tile_h=th, fwd_ppt=args.fwd_ppt, bwd_ppt=args.bwd_ppt, persistent=args.persistent,
             tile_cull=args.tile_cull)
    log(f"[bench] E16 = {E16:.4e} evals per step ({V} views, {P} pixels, {n} Gaussians)")

    tuned = None
    if args.autotune:
        batched_step()  # fills the image gradient the tuner backpropagates
        torch.cuda.synchronize()
        t_at = time.perf_counter()
        tuned, tune_ms = rast.autotune(frame, params, m_hard, cams, d_img, images=images, out=grads)
        log(f"[bench] autotune: {tuned} ({tune_ms:.3f} ms fwd+bwd) in {time.perf_counter() - t_at:.1f} s")
    # work counters of the settings actually timed (one untimed step), then
    # the timed configuration without counters
    rast.set(stats=1)
    batched_step()
    torch.cuda.synchronize()
    counts = rast.count_evals(frame)
    fstats = rast.stats(frame)
    rast.set(stats=0)
    for _ in range(args.warmup):
        batched_step()
    torch.cuda.synchronize()

    # per-stage profile: eager steps with HIP events around every stage on
    # the launch stream (a graph replay cannot be split by stage)
    M.mgs_profile_enable(ctx, True)
    n_prof = max(1, min(args.steps, 5))
    for _ in range(n_prof):
        batched_step()
    torch.cuda.synchronize()
    prof = M.mgs_profile_read(ctx)
    M.mgs_profile_enable(ctx, False)
    prof = {k: (v[0] / n_prof, v[1] // n_prof) for k, v in prof.items()}

    graph = None
    run = batched_step
    if args.graph:
        # fixed workspace, then capture one whole step into a hipGraph
        rast.reserve(frame, 1.25)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            batched_step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            batched_step()
        run = graph.replay
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        rast.check(frame)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    if graph is not None:
        rast.check(frame)  # raises if a replay outgrew the fixed workspace
        # the replayed step must equal an eager step on the same inputs
        img_g, dm_g, dp_g = images.clone(), grads.masks.clone(), grads.means.clone()
        batched_step()
        torch.cuda.synchronize()
        same_img = bool(torch.equal(img_g, images))
        e_m = float((dm_g - grads.masks).norm() / grads.masks.norm().clamp_min(1e-30))
        e_p = float((dp_g - grads.means).norm() / grads.means.norm().clamp_min(1e-30))
        if not same_img or e_m > 1e-5 or e_p > 1e-5:
            raise RuntimeError(f"graph replay differs from the eager step: images equal {same_img}, "
                               f"dM rel {e_m:.2e}, dmeans rel {e_p:.2e}")
    log(f"[bench] batched{' (graph)' if graph is not None else ''}: {ms_step:.3f} ms/step "
        f"(wall {1e3 * wall / args.steps:.3f}), K = {fstats['n_instances']}, wide records = {fstats['n_wide']}")
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    for k, v in prof.items():
        if v[1]:
            log(f"[bench]   {k:14s} {v[0] / v[1]:9.3f} ms/launch x {v[1]}")
    dom = max(stage_ms, key=lambda k: prof[k][0])
    roof = stage_roofline(dom, stage_ms[dom], counts, fstats, n, V, deg)
    roof = {"kernel": dom, "ms_per_launch": stage_ms[dom], **roof, "traffic": measured_traffic(dom)}

    plain = None
    if not args.no_plain and V > 1:
        rast_p = Rasterizer(0, sh_degree=deg, tile_w=16, tile_h=16, persistent=0)
        fr = rast_p.acquire_frame()
        offs = np.cumsum([0] + [3 * c["width"] * c["height"] for c in cams])

        def plain_step():
            M.mgs_sample_masks(rast_p.ctx, scores, tau, seed, step_id, m_hard, y_soft)
            for v, c in enumerate(cams):
                im = images[offs[v]:offs[v + 1]]
                dv = d_img[offs[v]:offs[v + 1]]
                rast_p.forward(fr, params, m_hard, [c], images=im)
                M.mgs_l1_loss_grad(rast_p.ctx, im, targets[offs[v]:offs[v + 1]], dv, loss, red_scratch)
                rast_p.backward(fr, params, dv, out=grads)
            M.mgs_mask_grad(rast_p.ctx, grads.masks, m_hard, y_soft, tau, lambda_m, d_scores, loss_m, red_scratch)

        for _ in range(max(1, args.warmup // 2)):
            plain_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.plain_steps):
            plain_step()
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / args.plain_steps
        plain = {"ms_per_step": pms, "evals_per_s": E16 / (pms * 1e-3), "views_per_s": V / (pms * 1e-3)}
        log(f"[bench] plain: {pms:.3f} ms/step")

    extras = None
    if not args.no_extras:
        extras = prune_and_render(rast, params, n, cams, seed)
        log(f"[bench] pruning: {extras['prune']['ms']:.3f} ms ({extras['prune']['kept']} of {n} kept, "
            f"{extras['prune']['GB_per_s']:.0f} GB/s); forward only: full {extras['render_only']['full']['ms']:.3f} ms, "
            f"pruned {extras['render_only']['pruned']['ms']:.3f} ms for {V} views "
            f"(x{extras['render_only']['speedup']:.2f}); with importance {extras['importance']['ms']:.3f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample of the views ...")
        cpu = cpu_baseline(scene, tau, seed, step_id)
        log(f"[bench] oracle: {cpu['sample']} on {cpu['cores']} threads")

    value = E16 / (ms_step * 1e-3)
    out = {
        "metric": "masked fwd+bwd Gaussian-pixel evals/s and views/s, batched vs plain, at oracle tol",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "gaussians": n,
            "views": V,
            "pixels": P,
            "evals_per_step_16x16": E16,
            "instances": fstats["n_instances"],
            "wide_records": fstats["n_wide"],
            "views_per_s": V / (ms_step * 1e-3),
            "tile": f"{rast.settings.tile_w}x{rast.settings.tile_h}",
            "batch_depth": rast.settings.batch_depth,
            "fwd_ppt": rast.settings.fwd_ppt,
            "bwd_ppt": rast.settings.bwd_ppt,
            "wide_tiles": rast.settings.wide_tiles,
            "tile_cull": bool(rast.settings.tile_cull),
            "autotuned": tuned is not None,
            "graph": graph is not None,
            "persistent": bool(rast.settings.persistent),
            "eval_counts": counts,
            "plain": plain,
            "pruning": extras["prune"] if extras else None,
            "render_only": extras["render_only"] if extras else None,
            "importance": extras["importance"] if extras else None,
            "stage_ms": {k: round(v, 4) for k, v in stage_ms.items() if prof[k][1]},
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
