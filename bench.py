#!/usr/bin/env python
"""Throughput of masked forward + backward rasterization on one MI355X.

A step is one pass of the hot path over one batch of synthetic input:
straight-through Gumbel mask sampling, projection, tile counts, scan, key
duplication, radix sort, tile ranges, masked compositing, L1 loss gradient,
masked backward compositing, projection backward and the mask-score
gradient.  The default workload is the batched multi-view case: a
1M-Gaussian unbounded scene (SH degree 3, heavy-tailed scales) rendered for
8 views of uneven size in one call ("batched"), compared with 8 single-view
calls of the same work ("plain").

metric: Gaussian-pixel evaluations per second, counting for every pixel the
sorted entries its 16x16 tile list presents up to and including its stop
entry (the forward evaluations; each has a backward counterpart).

Also reported (not the headline): the evaluated pairs per second, the
single-view workloads (tiny, object, unbounded), the 200-step training run of
the 3M-Gaussian workload (autograd step with Adam, captured per camera batch),
pruning and forward-only rendering, the FP64 oracle on the host cores, and an
oracle parity check of one view of the timed step.

Prints one JSON line.  --gpus N > 1 is rejected: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU lane-slots per Gaussian-pixel evaluation, counted from the formulas
# (each add, multiply, fused multiply-add, compare or select is one slot; exp
# and reciprocal issue at half rate on gfx950 and count two: a loop of
# independent exp2 + FMA pairs runs at 12.9 T pairs/s, 1 / (1 + 2) of the
# 39.3 T slot peak).
SLOTS_FILTER = 14      # dx, dy, Q, cut, exp, o*G, clamp, alpha filter
SLOTS_BLEND = 9        # M*a, test, stop compare, weight, 3 colour FMAs, T
SLOTS_BWD_VISIBLE = 42  # T recovery (rcp), X, dL/dM, dL/dc, dL/do, dL/dQ, dL/du,dv, conic, b update
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


def stage_work(stage: str, counts: dict, fs: dict, n: int, sh_deg: int, P: int):
    """Algorithmic (HBM bytes, VALU lane-slots) of one launch of a stage."""
    K = fs["n_instances"]
    R = fs["n_records"]
    k3 = 3 * (sh_deg + 1) ** 2
    if stage == "composite_fwd":
        slots = SLOTS_FILTER * counts["evaluated"] + SLOTS_BLEND * counts["blended"]
        # staged records, per-pixel outputs, and the clearing of the
        # backward's FP64 accumulator (9 doubles per record)
        return 48 * K + 20 * P + 72 * R, slots
    if stage == "composite_bwd":
        vis = counts["blended"] - counts["blended_masked"]
        slots = (SLOTS_FILTER * counts["bwd_evaluated"] + SLOTS_BWD_VISIBLE * vis +
                 SLOTS_BWD_MASKED * counts["blended_masked"])
        return 48 * K + 20 * P + 12 * P, slots
    if stage == "sort":
        # stable pass over 32-bit cell keys and 32-bit values: read and write both
        return 16 * K * fs["sort_passes"], 0
    if stage == "depth_sort":
        # 4 passes over 32-bit keys and values (read and written), then the
        # classification: order and key read, one record gathered (48 B),
        # the sorted copy (48 B), the count (wide flag in its top bit) and
        # the cull mask written
        return 16 * R * 4 + R * (8 + 48 + 48 + 4 + 8), 0
    if stage == "project":
        # parameters read once; record (48 B), depth, tile count, depth key
        # and order written per record
        return n * 4 * (11 + k3 + 1) + R * (48 + 4 * 4), 0
    if stage == "project_bwd":
        # parameters read, the FP64 gradient row (9 doubles) read per record,
        # parameter gradients written
        return n * 4 * (11 + k3) + R * 72 + n * 4 * (10 + k3), 0
    if stage == "duplicate":
        # per position: count, cull mask and the record's geometry (32 B); per
        # list entry a key and a value written
        return R * (4 + 8 + 32) + K * 8, 0
    if stage == "scan":
        # the list offsets: one count read and one 8-byte offset written per
        # wave of 64 positions
        return (R + 63) // 64 * 12, 0
    if stage == "ranges":
        return K * 4 + 8 * fs["total_tiles"], 0
    if stage == "sample_masks":
        return 16 * n, 0
    if stage == "mask_grad":
        return 24 * n, 0
    if stage == "loss":
        return 36 * P, 0
    return 0, 0


def stage_roofline(stage: str, ms_per_launch: float, counts: dict, fs: dict, n: int, sh_deg: int, P: int):
    """The roofline of the bound that limits a stage: VALU lane-slots for
    the compositing kernels, HBM bytes for the rest."""
    t = ms_per_launch * 1e-3
    byt, slots = stage_work(stage, counts, fs, n, sh_deg, P)
    if slots:
        return dict(bound="alu", achieved=slots / t / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                    frac=slots / t / PEAK_SLOTS, algorithmic=slots, algorithmic_unit="VALU lane-slots")
    return dict(bound="hbm", achieved=byt / t / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s", frac=byt / t / PEAK_HBM,
                algorithmic=byt, algorithmic_unit="bytes")


def combined_roofline(stage_ms: dict, counts: dict, fs: dict, n: int, sh_deg: int, P: int, ms_step: float):
    """t_roof = sum over stages of max(bytes / HBM peak, slots / VALU peak),
    against the measured step; plus each stage's own fraction."""
    t_roof, per = 0.0, {}
    for st, ms in stage_ms.items():
        byt, slots = stage_work(st, counts, fs, n, sh_deg, P)
        t = max(byt / PEAK_HBM, slots / PEAK_SLOTS)
        t_roof += t
        if ms > 0:
            per[st] = {"ms": round(ms, 4), "roof_ms": round(1e3 * t, 4), "frac": round(1e3 * t / ms, 3),
                       "bound": "alu" if slots / PEAK_SLOTS > byt / PEAK_HBM else "hbm"}
    return {"t_roof_ms": 1e3 * t_roof, "ms_per_step": ms_step, "frac": 1e3 * t_roof / ms_step, "stages": per}


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


def host_cpu() -> dict:
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


# ---------------------------------------------------------------------------
# one workload: the step, its evaluation count, its timing and roofline
# ---------------------------------------------------------------------------

class Workload:
    """Device inputs and buffers of one workload and its batched step."""

    def __init__(self, scene: dict, desc: str, settings: dict, lambda_m: float = 0.1, seed: int = 2412,
                 step_id: int = 0):
        import torch
        from paper_2412_20522_amd import maskgs as M
        from paper_2412_20522_amd.raster import PARAM_KEYS, Grads, Rasterizer
        self.M, self.torch = M, torch
        self.scene, self.desc = scene, desc
        self.cams = scene["cameras"]
        self.V = len(self.cams)
        self.n = scene["means"].shape[0]
        self.deg = scene["sh_degree"]
        self.tau = float(scene.get("gumbel_tau", 0.5))
        self.lambda_m, self.seed, self.step_id = lambda_m, seed, step_id
        dev = torch.device("cuda:0")
        self.params = {k: torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).to(dev) for k in PARAM_KEYS}
        self.scores = torch.from_numpy(np.ascontiguousarray(scene["mask_scores"], np.float32)).to(dev)
        self.P = sum(c["width"] * c["height"] for c in self.cams)
        self.targets = torch.cat([torch.from_numpy(t.reshape(-1)) for t in scene["targets"]]).to(dev)
        self.rast = Rasterizer(0, sh_degree=self.deg, **settings)
        self.frame = self.rast.acquire_frame()
        self.images = torch.empty(3 * self.P, device=dev)
        self.d_img = torch.empty_like(self.images)
        self.loss = torch.zeros(1, device=dev)
        self.loss_m = torch.zeros(1, device=dev)
        self.grads = Grads(*(torch.empty_like(self.params[k]) for k in PARAM_KEYS), torch.empty(self.n, device=dev))
        self.d_scores = torch.empty(self.n, 2, device=dev)
        self.m_hard = torch.empty(self.n, device=dev)
        self.y_soft = torch.empty(self.n, device=dev)
        self.red = torch.empty(int(M.lib().mgs_reduce_scratch_bytes(3 * self.P)), dtype=torch.uint8, device=dev)

    def step(self):
        M, r = self.M, self.rast
        M.mgs_sample_masks(r.ctx, self.scores, self.tau, self.seed, self.step_id, self.m_hard, self.y_soft)
        r.forward(self.frame, self.params, self.m_hard, self.cams, images=self.images)
        M.mgs_l1_loss_grad(r.ctx, self.images, self.targets, self.d_img, self.loss, self.red)
        r.backward(self.frame, self.params, self.d_img, out=self.grads)
        M.mgs_mask_grad(r.ctx, self.grads.masks, self.m_hard, self.y_soft, self.tau, self.lambda_m, self.d_scores,
                        self.loss_m, self.red)

    def settings_dict(self) -> dict:
        st = self.rast.settings
        return {k: getattr(st, k) for k in ("tile_w", "tile_h", "batch_depth", "fwd_ppt", "bwd_ppt", "wide_tiles",
                                           "tile_cull")}


def measure(w: Workload, steps: int, warmup: int, autotune: bool, graph: bool, label: str) -> dict:
    """E16 at 16x16 tiles (untimed), optional autotuning, work counters, a
    per-stage profile of eager steps, then `steps` graph replays timed with
    HIP events on the launch stream, checked against an eager step."""
    torch, M, rast = w.torch, w.M, w.rast
    timed = w.settings_dict()
    # the evaluation count at 16x16 tiles on the lists of Sec. 3.1 exactly
    # (no culling), whatever the timed configuration skips
    rast.set(tile_w=16, tile_h=16, fwd_ppt=1, bwd_ppt=4, persistent=0, tile_cull=0, stats=1)
    M.mgs_sample_masks(rast.ctx, w.scores, w.tau, w.seed, w.step_id, w.m_hard, w.y_soft)
    rast.forward(w.frame, w.params, w.m_hard, w.cams, images=w.images)
    E16 = rast.count_evals(w.frame)["examined"]
    rast.set(persistent=1, **timed)
    log(f"[bench] {label}: E16 = {E16:.4e} evals per step ({w.V} views, {w.P} pixels, {w.n} Gaussians)")
    tuned = None
    if autotune:
        w.step()  # fills the image gradient the tuner backpropagates
        torch.cuda.synchronize()
        t_at = time.perf_counter()
        tuned, tune_ms = rast.autotune(w.frame, w.params, w.m_hard, w.cams, w.d_img, images=w.images, out=w.grads)
        log(f"[bench] {label}: autotune {tuned} ({tune_ms:.3f} ms fwd+bwd) in {time.perf_counter() - t_at:.1f} s")
    # work counters of the settings actually timed (one untimed step), then
    # the timed configuration without counters
    rast.set(stats=1)
    w.step()
    torch.cuda.synchronize()
    counts = rast.count_evals(w.frame)
    fstats = rast.stats(w.frame)
    rast.set(stats=0)
    for _ in range(warmup):
        w.step()
    torch.cuda.synchronize()
    # per-stage profile: eager steps with HIP events around every stage on
    # the launch stream (a graph replay cannot be split by stage)
    M.mgs_profile_enable(rast.ctx, True)
    n_prof = max(1, min(steps, 5))
    for _ in range(n_prof):
        w.step()
    torch.cuda.synchronize()
    prof = M.mgs_profile_read(rast.ctx)
    M.mgs_profile_enable(rast.ctx, False)
    stage_ms = {k: v[0] / v[1] for k, v in prof.items() if v[1]}
    g = None
    run = w.step
    if graph:
        rast.reserve(w.frame, 1.25)  # fixed workspace, then one whole step captured
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            w.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            w.step()
        run = g.replay
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        rast.check(w.frame)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / steps
    if g is not None:
        rast.check(w.frame)  # raises if a replay outgrew the fixed workspace
        # the replayed step must equal an eager step on the same inputs
        img_g, dm_g, dp_g = w.images.clone(), w.grads.masks.clone(), w.grads.means.clone()
        w.step()
        torch.cuda.synchronize()
        same_img = bool(torch.equal(img_g, w.images))
        e_m = float((dm_g - w.grads.masks).norm() / w.grads.masks.norm().clamp_min(1e-30))
        e_p = float((dp_g - w.grads.means).norm() / w.grads.means.norm().clamp_min(1e-30))
        if not same_img or e_m > 1e-5 or e_p > 1e-5:
            raise RuntimeError(f"graph replay differs from the eager step: images equal {same_img}, "
                               f"dM rel {e_m:.2e}, dmeans rel {e_p:.2e}")
    log(f"[bench] {label}{' (graph)' if g is not None else ''}: {ms_step:.3f} ms/step "
        f"(wall {1e3 * wall / steps:.3f}), K = {fstats['n_instances']}, wide records = {fstats['n_wide']}")
    for k, v in stage_ms.items():
        log(f"[bench]   {k:14s} {v:9.3f} ms/launch")
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    roof = stage_roofline(dom, stage_ms[dom], counts, fstats, w.n, w.deg, w.P)
    roof = {"kernel": dom, "ms_per_launch": stage_ms[dom], **roof}
    comb = combined_roofline(stage_ms, counts, fstats, w.n, w.deg, w.P, ms_step)
    return {"E16": E16, "ms_per_step": ms_step, "counts": counts, "fstats": fstats, "stage_ms": stage_ms,
            "roofline": roof, "combined": comb, "tuned": tuned, "graph": g}


def plain_path(w: Workload, reps: int, warmup: int, autotune: bool) -> dict:
    """The same step as 8 single-view calls: one forward and backward per
    view, no graph and no persistent queue, no counters.  The compositing
    settings are the autotuner's for each view (autotune) or the batched
    path's tuned ones.  The L1 gradient of each view is weighted by
    its share of the elements (so the per-view losses add up to the mean over
    all views) and the per-view parameter gradients are summed by the library
    (accumulating backward), so the step computes what the batched step
    does; checked once."""
    torch, M = w.torch, w.M
    from paper_2412_20522_amd.raster import PARAM_KEYS, Grads, Rasterizer
    st = w.settings_dict()
    rp = Rasterizer(0, sh_degree=w.deg, persistent=0, stats=0, **st)
    fr = rp.acquire_frame()
    per_view = [rp.settings] * w.V
    if autotune:
        M.mgs_sample_masks(rp.ctx, w.scores, w.tau, w.seed, w.step_id, w.m_hard, w.y_soft)
        base = rp.settings
        per_view = []
        off = 0
        for cam in w.cams:
            rp.settings = base
            im = rp.forward(fr, w.params, w.m_hard, [cam])
            d1 = torch.empty_like(im)
            M.mgs_l1_loss_grad(rp.ctx, im, w.targets[off:off + im.numel()], d1, None, w.red)
            off += im.numel()
            rp.autotune(fr, w.params, w.m_hard, [cam], d1, images=im)
            per_view.append(rp.settings)
        st = [{k: getattr(x, k) for k in st} for x in per_view]
    offs = np.cumsum([0] + [3 * c["width"] * c["height"] for c in w.cams])
    m_tot = float(offs[-1])
    scale = [torch.full((1,), float(offs[v + 1] - offs[v]) / m_tot, device="cuda") for v in range(w.V)]
    grads = Grads(*(torch.empty_like(w.params[k]) for k in PARAM_KEYS), torch.empty(w.n, device="cuda"))
    d_scores = torch.empty_like(w.d_scores)
    images = torch.empty_like(w.images)
    d_img = torch.empty_like(w.d_img)
    loss_v = torch.zeros(1, device="cuda")
    m_hard, y_soft = torch.empty_like(w.m_hard), torch.empty_like(w.y_soft)

    def plain_step():
        M.mgs_sample_masks(rp.ctx, w.scores, w.tau, w.seed, w.step_id, m_hard, y_soft)
        for v, c in enumerate(w.cams):
            im = images[offs[v]:offs[v + 1]]
            dv = d_img[offs[v]:offs[v + 1]]
            rp.settings = per_view[v]
            rp.forward(fr, w.params, m_hard, [c], images=im)
            M.mgs_l1_loss_grad(rp.ctx, im, w.targets[offs[v]:offs[v + 1]], dv, loss_v, w.red, grad_scale=scale[v])
            rp.backward(fr, w.params, dv, out=grads, accumulate=v > 0)
        M.mgs_mask_grad(rp.ctx, grads.masks, m_hard, y_soft, w.tau, w.lambda_m, d_scores, None, w.red)

    for _ in range(max(1, warmup)):
        plain_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plain_step()
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / reps
    # the same result as the batched step
    w.step()
    torch.cuda.synchronize()
    same = {"images_equal": bool(torch.equal(images, w.images))}
    for k in PARAM_KEYS + ("masks",):
        a, b = getattr(grads, k), getattr(w.grads, k)
        same[k] = float((a - b).norm() / b.norm().clamp_min(1e-30))
    same["mask_scores"] = float((d_scores - w.d_scores).norm() / w.d_scores.norm().clamp_min(1e-30))
    same["ok"] = bool(same["images_equal"] and max(v for k, v in same.items() if k != "images_equal") <= 1e-5)
    if not same["ok"]:
        log(f"[bench] the plain path's step differs from the batched step: {same}")
    rp.release_frame(fr)
    return {"ms_per_step": pms, "views_per_s": w.V / (pms * 1e-3),
            "settings": st if isinstance(st, list) else {**st, "persistent": 0, "stats": 0},
            "same_result_as_batched": same}


# ---------------------------------------------------------------------------
# oracle legs (host cores; outside every timed region)
# ---------------------------------------------------------------------------

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
            "views_per_s": len(done) / dt, "seconds": dt, **host_cpu()}


def parity_check(w: Workload, view: int = 0) -> dict:
    """The timed step's image of one view against the oracle run on the
    GPU's own projected records of that view (stage protocol): element-wise
    on the pixels whose discrete decisions are away from their thresholds."""
    import oracle
    torch, M = w.torch, w.M
    ex = {k: M.mgs_frame_export(w.rast.ctx, w.frame, k) for k in ("records", "radius", "depth")}
    torch.cuda.synchronize()
    n = w.n
    rec = ex["records"].view(-1, 12)[view * n:(view + 1) * n].cpu().numpy().astype(np.float64)
    rad = ex["radius"][view * n:(view + 1) * n].cpu().numpy().astype(np.float64)
    dbits = ex["depth"][view * n:(view + 1) * n].cpu().numpy().view(np.uint32)
    a, beta, gamma = rec[:, 2], rec[:, 3], rec[:, 4]
    conic = np.stack([a, a * beta, gamma + (a * beta) * beta], 1)
    cam = w.cams[view]
    ost = oracle.RasterSettings(sh_degree=w.deg)
    masks = w.m_hard.cpu().numpy().astype(np.float64)
    lists = oracle.build_lists([cam["width"]], [cam["height"]], n, rec[:, 0:2], rad, dbits,
                               (rad > 0).astype(np.uint8), ost)
    of = oracle.render_fwd([cam["width"]], [cam["height"]], n, rec[:, 0:2], conic, rec[:, 5], rec[:, 8:11], masks,
                           lists, ost)
    p = cam["width"] * cam["height"]
    img = w.images[:3 * p].cpu().numpy().astype(np.float64)
    ok = np.tile(of.flags == 0, 3)
    scale = max(float(np.abs(of.image).max()), 1.0)
    err = float(np.abs(img - of.image)[ok].max())
    return {"view": f"{cam['width']}x{cam['height']}", "pixels": p, "flagged_fraction": float(1 - ok.mean()),
            "max_abs_err_unflagged": err, "tolerance": 1e-5 * scale, "ok": bool(err <= 1e-5 * scale),
            "protocol": "oracle compositing on the GPU's own records of the timed step"}


# ---------------------------------------------------------------------------
# extras: pruning, forward-only rendering, training
# ---------------------------------------------------------------------------

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
        rast.reserve(fr, 0)
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


def training_run(n: int, steps: int, lambda_m: float, settings: dict, oracle_eval: bool = True,
                 batch: int = 4, seed: int = 5) -> dict:
    """The training workload: targets rendered from the ground-truth set
    (all masks 1) at 32 poses, then `steps` steps of the autograd training
    step (Gumbel masks, masked forward, L1 + lambda_m L_m, backward, Adam on
    every attribute and both scores) in batches of 4 views, each batch's step
    captured once into a hipGraph.  Reports ms per step, the trajectory of the
    sampled mask fraction and of the L1 loss, and the PSNR on the 128x128
    evaluation crop of view 0 against the ground truth, rendered by the GPU
    and by the FP64 oracle (masks from 10 pruning draws)."""
    import torch
    import scenegen
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import PARAM_KEYS, Rasterizer
    from paper_2412_20522_amd.train import TRAIN_KEYS, Trainer
    t_gen = time.perf_counter()
    ts = scenegen.training_scene(n=n)
    gt, tr, cams = ts["gt"], ts["trainee"], ts["cameras"]
    log(f"[bench] training: generated {ts['name']} in {time.perf_counter() - t_gen:.1f} s")
    dev = torch.device("cuda:0")
    rast = Rasterizer(0, sh_degree=3, bg=(0.0, 0.0, 0.0), persistent=1, stats=0, **settings)
    batches = [cams[i:i + batch] for i in range(0, len(cams), batch)]
    gtp = {k: torch.from_numpy(np.ascontiguousarray(gt[k], np.float32)).to(dev) for k in PARAM_KEYS}
    ones = torch.ones(n, device=dev)
    fr = rast.acquire_frame()
    targets = [rast.forward(fr, gtp, ones, b).clone() for b in batches]
    params = {k: torch.from_numpy(np.ascontiguousarray(tr[k], np.float32)).to(dev) for k in TRAIN_KEYS}
    crop = scenegen.crop_camera(cams[0], 896, 480, 128, 128)
    gt_crop = rast.forward(fr, gtp, ones, [crop]).clone()
    eval_seed = 777

    def evaluate(label: str) -> dict:
        keep = torch.empty(n, dtype=torch.int32, device=dev)
        M.mgs_prune_sample(rast.ctx, params["mask_scores"].detach(), eval_seed, 0, 10, keep)
        m_eval = keep.to(torch.float32)
        img = rast.forward(fr, {k: params[k].detach() for k in PARAM_KEYS}, m_eval, [crop]).clone()
        torch.cuda.synchronize()
        out = {"kept_fraction": float(m_eval.mean()),
               "psnr_gpu": float(-10 * torch.log10(((img - gt_crop) ** 2).mean()))}
        if oracle_eval:
            import oracle
            host = {k: params[k].detach().cpu().numpy() for k in TRAIN_KEYS}
            mk = oracle.prune_keep(host["mask_scores"], eval_seed, 0, 10).astype(np.float64)
            ost = oracle.RasterSettings(sh_degree=3)
            o_img = oracle.run_pipeline(host, [crop], mk, ost, backward=False).fwd.image
            o_gt = oracle.run_pipeline(gt, [crop], np.ones(n), ost, backward=False).fwd.image
            g_img = img.cpu().numpy().astype(np.float64)
            out["psnr_oracle"] = oracle.psnr(o_img, o_gt)
            out["masks_equal_oracle"] = bool(np.array_equal(mk, m_eval.cpu().numpy().astype(np.float64)))
            out["gpu_vs_oracle_max_abs"] = float(np.abs(g_img - o_img).max())
            out["gpu_vs_oracle_psnr"] = oracle.psnr(g_img, o_img)
        log(f"[bench] training {label}: {out}")
        return out

    before = evaluate("before")
    trainer = Trainer(rast, params, batches, targets, tau=0.5, seed=seed, lambda_m=lambda_m)
    t_prep = time.perf_counter()
    trainer.reserve(1.5)
    warm = 3
    hist_l1 = torch.zeros(steps, device=dev)
    hist_lm = torch.zeros(steps, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for i in range(warm):
            rec = trainer.step()
            hist_l1[i].copy_(rec.l1)
            hist_lm[i].copy_(rec.mask_loss)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    trainer.capture()
    log(f"[bench] training: reserved and captured {len(batches)} graphs in {time.perf_counter() - t_prep:.1f} s")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(warm, steps):
        rec = trainer.step()
        hist_l1[i].copy_(rec.l1)
        hist_lm[i].copy_(rec.mask_loss)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(steps - warm, 1)
    trainer.check()
    after = evaluate("after")
    l1 = hist_l1.cpu().numpy()
    frac = np.sqrt(hist_lm.cpu().numpy())  # L_m = (mean M)^2
    pick = sorted(set(list(range(0, steps, 10)) + [steps - 1]))
    sc = params["mask_scores"].detach()
    p_exist = float(torch.sigmoid(sc[:, 0] - sc[:, 1]).mean())
    trainer.close()
    rast.release_frame(fr)
    return {"gaussians": n, "views_per_step": batch, "view_size": f"{cams[0]['width']}x{cams[0]['height']}",
            "poses": len(cams), "steps": steps, "lambda_m": lambda_m, "graphs": len(batches),
            "ms_per_step": ms, "views_per_s": batch / (ms * 1e-3),
            "timed": f"{steps - warm} graph replays after {warm} eager steps",
            "sampled_mask_fraction": {str(i): round(float(frac[i]), 5) for i in pick},
            "l1": {str(i): round(float(l1[i]), 5) for i in pick},
            "mean_existence_probability_end": p_exist,
            "crop_eval": {"crop": "view 0, origin (896, 480), 128x128", "before": before, "after": after}}


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
    ap.add_argument("--no-single-view", action="store_true", help="skip the single-view workloads")
    ap.add_argument("--train-steps", type=int, default=200, help="training run length (0: skip it)")
    ap.add_argument("--train-gaussians", type=int, default=3_000_000)
    ap.add_argument("--train-lambda", type=float, default=0.1)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--batch-depth", type=int, default=128)
    ap.add_argument("--fwd-ppt", type=int, default=2)
    ap.add_argument("--bwd-ppt", type=int, default=4)
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
    tw, th = (int(x) for x in args.tile.split("x"))
    base = dict(tile_w=tw, tile_h=th, batch_depth=args.batch_depth, fwd_ppt=args.fwd_ppt, bwd_ppt=args.bwd_ppt,
                wide_tiles=args.wide_tiles, tile_cull=args.tile_cull)
    w = Workload(scene, desc, dict(base, persistent=1))
    res = measure(w, args.steps, args.warmup, bool(args.autotune), bool(args.graph), args.workload)
    ms_step, E16, counts, fstats = res["ms_per_step"], res["E16"], res["counts"], res["fstats"]
    tuned = w.settings_dict()
    roof = dict(res["roofline"])
    roof["traffic"] = measured_traffic(roof["kernel"])
    roof["combined"] = res["combined"]

    plain = None
    if not args.no_plain and w.V > 1:
        plain = plain_path(w, args.plain_steps, max(1, args.warmup // 2), autotune=bool(args.autotune))
        log(f"[bench] plain: {plain['ms_per_step']:.3f} ms/step with {plain['settings']}, "
            f"same result: {plain['same_result_as_batched']}")
        if args.autotune:
            alt = plain_path(w, args.plain_steps, max(1, args.warmup // 2), autotune=False)
            plain["with_batched_settings"] = {k: alt[k] for k in ("ms_per_step", "views_per_s", "settings")}
            log(f"[bench] plain with the batched settings: {alt['ms_per_step']:.3f} ms/step")

    extras = None
    if not args.no_extras:
        extras = prune_and_render(w.rast, w.params, w.n, w.cams, w.seed)
        log(f"[bench] pruning: {extras['prune']['ms']:.3f} ms ({extras['prune']['kept']} of {w.n} kept, "
            f"{extras['prune']['GB_per_s']:.0f} GB/s); forward only: full {extras['render_only']['full']['ms']:.3f} ms, "
            f"pruned {extras['render_only']['pruned']['ms']:.3f} ms for {w.V} views "
            f"(x{extras['render_only']['speedup']:.2f}); with importance {extras['importance']['ms']:.3f} ms")

    single = None
    if not args.no_single_view and args.workload == "batched":
        single = {}
        for name in ("tiny", "object", "unbounded"):
            sc, d = build_workload(name)
            ws = Workload(sc, d, dict(base, persistent=1))
            r = measure(ws, args.steps, args.warmup, bool(args.autotune), bool(args.graph), name)
            single[name] = {"workload": d, "ms_per_step": r["ms_per_step"], "evals_per_step_16x16": r["E16"],
                            "evals_per_s": r["E16"] / (r["ms_per_step"] * 1e-3),
                            "evaluated_pairs_per_s": r["counts"]["evaluated"] / (r["ms_per_step"] * 1e-3),
                            "views_per_s": 1.0 / (r["ms_per_step"] * 1e-3), "settings": ws.settings_dict(),
                            "roofline": {k: r["roofline"][k] for k in ("kernel", "bound", "frac", "ms_per_launch")},
                            "combined_frac": r["combined"]["frac"],
                            "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()}}
            ws.rast.reserve(ws.frame, 0)
            ws.rast.release_frame(ws.frame)
            del ws

    training = None
    if args.train_steps > 0 and args.workload == "batched":
        training = training_run(args.train_gaussians, args.train_steps, args.train_lambda,
                                {k: tuned[k] for k in ("tile_w", "tile_h", "batch_depth", "fwd_ppt", "bwd_ppt",
                                                       "wide_tiles", "tile_cull")},
                                oracle_eval=not args.no_cpu_baseline)
        log(f"[bench] training: {training['ms_per_step']:.3f} ms/step")

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        parity = parity_check(w, 0)
        log(f"[bench] parity of the timed step (view {parity['view']}): {parity}")
        log("[bench] timing the FP64 oracle on a bounded sample of the views ...")
        cpu = cpu_baseline(scene, w.tau, w.seed, w.step_id)
        log(f"[bench] oracle: {cpu['sample']} on {cpu['cores']} threads ({cpu['cpu_model']}, nproc {cpu['nproc']})")

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
            "gaussians": w.n,
            "views": w.V,
            "pixels": w.P,
            "evals_per_step_16x16": E16,
            "evaluated_pairs_per_step": counts["evaluated"],
            "evaluated_pairs_per_s": counts["evaluated"] / (ms_step * 1e-3),
            "instances": fstats["n_instances"],
            "wide_records": fstats["n_wide"],
            "views_per_s": w.V / (ms_step * 1e-3),
            "tile": f"{tuned['tile_w']}x{tuned['tile_h']}",
            "batch_depth": tuned["batch_depth"],
            "fwd_ppt": tuned["fwd_ppt"],
            "bwd_ppt": tuned["bwd_ppt"],
            "wide_tiles": tuned["wide_tiles"],
            "tile_cull": bool(tuned["tile_cull"]),
            "autotuned": res["tuned"] is not None,
            "graph": res["graph"] is not None,
            "persistent": True,
            "eval_counts": counts,
            "plain": plain,
            "parity": parity,
            "single_view": single,
            "training": training,
            "pruning": extras["prune"] if extras else None,
            "render_only": extras["render_only"] if extras else None,
            "importance": extras["importance"] if extras else None,
            "stage_ms": {k: round(v, 4) for k, v in res["stage_ms"].items()},
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if parity is not None and not parity["ok"]:
        log("[bench] the timed step failed its parity check")
        print(json.dumps(out), flush=True)
        return 1
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
