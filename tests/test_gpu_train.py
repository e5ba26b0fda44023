"""The differentiable training step (autograd Functions, multi-array Adam,
device step counter) against the FP64 oracle, and its hipGraph capture.

- MaskedRasterize + L1Loss give the results of the plain library calls.
- A captured autograd forward + backward replays bit for bit (images) and to
  atomics reordering (gradients), with eager work between replays.
- One full training step on the 128x128 evaluation crop of the training
  workload: masks bit for bit, images and every gradient element-wise on
  unflagged pixels / Gaussians against the oracle run on the GPU's own
  records, and the Adam update element-wise against the oracle's Adam.
- The multi-array Adam with a device step counter matches the oracle's Adam
  over several steps; a captured training step advances the counter.
- Without a backward (no_grad) the pooled frame goes back to the pool.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TRAIN_KEYS = U.PARAM_KEYS + ("mask_scores",)


def _scene_views():
    s = scenegen.small_scene(2500, 96, 80, seed=401, sh_degree=2, log_scale_mean=-2.4, n_views=3)
    s["cameras"][1] = scenegen.orbit_camera(4.0, 40.0, 5.0, 72, 64)
    s["cameras"][2] = scenegen.orbit_camera(4.0, -70.0, 10.0, 50, 45)
    return s


def _leaves(s):
    return {k: torch.from_numpy(np.ascontiguousarray(s[k], np.float32)).cuda().requires_grad_(True)
            for k in TRAIN_KEYS}


def _targets(cams, seed):
    P = sum(c["width"] * c["height"] for c in cams)
    return torch.from_numpy(np.random.default_rng(seed).uniform(0, 1, 3 * P).astype(np.float32)).cuda()


def _autograd_step(rast, leaves, cams, tgt, tau, seed, lam, frame=None, counter=None):
    from paper_2412_20522_amd.raster import L1Loss, MaskedRasterize
    for t in leaves.values():
        t.grad = None
    images, lm = MaskedRasterize.apply(leaves["means"], leaves["log_scales"], leaves["quats"],
                                       leaves["opacity_logits"], leaves["sh"], leaves["mask_scores"], rast, cams,
                                       tau, seed, 0, frame, counter)
    l1 = L1Loss.apply(images, tgt, rast)
    (l1 + lam * lm).backward()
    return images.detach(), l1.detach(), lm.detach()


def test_autograd_step_equals_library_calls():
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import PARAM_KEYS, Rasterizer
    s = _scene_views()
    cams = s["cameras"]
    rast = Rasterizer(0, sh_degree=2, bg=(0.1, 0.2, 0.3))
    leaves = _leaves(s)
    tgt = _targets(cams, 1)
    tau, seed, lam = 0.5, 31, 0.3
    counter = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    images, l1, lm = _autograd_step(rast, leaves, cams, tgt, tau, seed, lam, counter=counter)
    torch.cuda.synchronize()
    # the same step through the plain entry points (mask step 5 = 0 + counter)
    n = s["means"].shape[0]
    params = {k: leaves[k].detach() for k in PARAM_KEYS}
    m = torch.empty(n, device="cuda")
    y = torch.empty(n, device="cuda")
    M.mgs_sample_masks(rast.ctx, leaves["mask_scores"].detach(), tau, seed, 5, m, y)
    assert torch.equal(m, rast.last_masks)
    frame = rast.acquire_frame()
    img2 = rast.forward(frame, params, m, cams)
    d_img = torch.empty_like(img2)
    loss = torch.zeros(1, device="cuda")
    M.mgs_l1_loss_grad(rast.ctx, img2, tgt, d_img, loss)
    g = rast.backward(frame, params, d_img)
    d_scores = torch.empty(n, 2, device="cuda")
    loss_m = torch.zeros(1, device="cuda")
    M.mgs_mask_grad(rast.ctx, g.masks, m, y, tau, lam, d_scores, loss_m)
    torch.cuda.synchronize()
    rast.release_frame(frame)
    assert torch.equal(images, img2)
    assert float(l1) == float(loss[0])
    assert float(lm) == float(loss_m[0])
    mh = m.cpu().numpy().astype(np.float64)
    assert float(lm) == pytest.approx((mh.mean()) ** 2, rel=1e-6)
    for k, ref in [("means", g.means), ("log_scales", g.log_scales), ("quats", g.quats),
                   ("opacity_logits", g.opacity_logits), ("sh", g.sh), ("mask_scores", d_scores)]:
        e = U.rel_err(leaves[k].grad.cpu().numpy(), ref.cpu().numpy())
        assert e <= 1e-6, (k, e)


def test_autograd_capture_replays_match_eager():
    from paper_2412_20522_amd.raster import Rasterizer
    s = _scene_views()
    cams = s["cameras"]
    rast = Rasterizer(0, sh_degree=2, bg=(0.1, 0.2, 0.3), persistent=1)
    leaves = _leaves(s)
    tgt = _targets(cams, 2)
    tau, seed, lam = 0.5, 32, 0.1
    counter = torch.full((1,), 3, dtype=torch.int64, device="cuda")
    frame = rast.acquire_frame()
    try:
        ref_img, _, _ = _autograd_step(rast, leaves, cams, tgt, tau, seed, lam, frame, counter)
        torch.cuda.synchronize()
        ref_img = ref_img.cpu().numpy()
        ref_g = {k: leaves[k].grad.cpu().numpy() for k in TRAIN_KEYS}
        rast.reserve(frame, 1.25)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _autograd_step(rast, leaves, cams, tgt, tau, seed, lam, frame, counter)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        for t in leaves.values():
            t.grad = None
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            img_c, l1_c, lm_c = _autograd_step(rast, leaves, cams, tgt, tau, seed, lam, frame, counter)
        grads_c = {k: leaves[k].grad for k in TRAIN_KEYS}
        torch.cuda.synchronize()
        for rep in range(3):
            img_c.fill_(-3.0 - rep)
            for t in grads_c.values():
                t.fill_(77.0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            rast.check(frame)
            assert np.array_equal(img_c.cpu().numpy(), ref_img), rep
            for k in TRAIN_KEYS:
                e = U.rel_err(grads_c[k].cpu().numpy(), ref_g[k])
                assert e <= 1e-6, (rep, k, e)
            _ = (img_c * 3.0).sum().item()  # eager work between replays
        del graph
    finally:
        rast.reserve(frame, 0)
        rast.release_frame(frame)


def test_no_grad_forward_returns_pooled_frame():
    from paper_2412_20522_amd.raster import MaskedRasterize, Rasterizer
    s = _scene_views()
    rast = Rasterizer(0, sh_degree=2)
    leaves = _leaves(s)
    fr = rast.acquire_frame()
    rast.release_frame(fr)
    assert len(rast._free_frames) == 1
    for _ in range(3):
        with torch.no_grad():
            img, lm = MaskedRasterize.apply(leaves["means"], leaves["log_scales"], leaves["quats"],
                                            leaves["opacity_logits"], leaves["sh"], leaves["mask_scores"], rast,
                                            s["cameras"], 0.5, 1, 0)
        torch.cuda.synchronize()
        assert len(rast._free_frames) == 1
    # a graph dropped without a backward also gives its frame back
    img, lm = MaskedRasterize.apply(leaves["means"], leaves["log_scales"], leaves["quats"], leaves["opacity_logits"],
                                    leaves["sh"], leaves["mask_scores"], rast, s["cameras"], 0.5, 1, 0)
    assert len(rast._free_frames) == 0
    del img, lm
    assert len(rast._free_frames) == 1


def test_adam_multi_matches_oracle_with_device_step():
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import Rasterizer
    rast = Rasterizer(0)
    rng = np.random.default_rng(9)
    sizes = [1, 3, 4097, 70_001, 12, 0, 16 * 256 * 4 + 5]
    lrs = [1e-2, 5e-3, 1e-3, 0.05, 2.5e-3, 1.0, 1e-4]
    P = [rng.normal(size=n).astype(np.float32) for n in sizes]
    dev = [dict(p=torch.from_numpy(p.copy()).cuda(), m=torch.zeros(len(p), device="cuda"),
                v=torch.zeros(len(p), device="cuda")) for p in P]
    host = [dict(p=p.astype(np.float64), m=np.zeros(len(p)), v=np.zeros(len(p))) for p in P]
    counter = torch.full((1,), 2, dtype=torch.int64, device="cuda")
    for it in range(4):
        G = [(rng.normal(size=n) * 10.0 ** rng.integers(-6, 1)).astype(np.float32) for n in sizes]
        gd = [torch.from_numpy(g).cuda() for g in G]
        M.mgs_adam_step_multi(rast.ctx, [(d["p"], g, d["m"], d["v"], lr) for d, g, lr in zip(dev, gd, lrs)],
                              0.9, 0.999, 1e-15, 1, step_offset=counter)
        M.mgs_step_advance(rast.ctx, counter, 1)
        for h, g, lr in zip(host, G, lrs):
            if h["p"].size:
                oracle.adam(h["p"], g.astype(np.float64), h["m"], h["v"], lr, 0.9, 0.999, 1e-15, 3 + it)
        torch.cuda.synchronize()
        for d, h, lr in zip(dev, host, lrs):
            p = d["p"].cpu().numpy().astype(np.float64)
            # each step moves a parameter by at most about lr: FP32 rounding of that
            assert np.all(np.abs(p - h["p"]) <= 2e-6 * (np.abs(h["p"]) + lr)), it
    assert int(counter.item()) == 6


def _crop_workload(n=48_000):
    ts = scenegen.training_scene(n=n, n_poses=2)
    crop = scenegen.crop_camera(ts["cameras"][0], 896, 480, 128, 128)
    return ts, crop


def test_training_step_matches_oracle_on_crop():
    """One full step of the training workload (Sec. 3.3-3.5; L1 + lambda_m
    L_m, Adam) on the 128x128 evaluation crop, element-wise against the
    oracle."""
    from paper_2412_20522_amd import maskgs as M
    from paper_2412_20522_amd.raster import Rasterizer
    from paper_2412_20522_amd.train import Trainer
    ts, crop = _crop_workload()
    gt, tr = ts["gt"], ts["trainee"]
    n = tr["means"].shape[0]
    ost = oracle.RasterSettings(sh_degree=3, bg=(0.0, 0.0, 0.0))
    target = oracle.run_pipeline(gt, [crop], np.ones(n), ost, backward=False).fwd.image.astype(np.float32)
    tau, seed, lam = 0.5, 2024, 0.1
    rast = Rasterizer(0, sh_degree=3, bg=(0.0, 0.0, 0.0))
    params = {k: torch.from_numpy(np.ascontiguousarray(tr[k], np.float32)).cuda() for k in TRAIN_KEYS}
    before = {k: tr[k].astype(np.float64).copy() for k in TRAIN_KEYS}
    trainer = Trainer(rast, params, [[crop]], [torch.from_numpy(target).cuda()], tau=tau, seed=seed, lambda_m=lam)
    rec = trainer.step(0)
    torch.cuda.synchronize()
    img = trainer.last_images.cpu().numpy().astype(np.float64)
    g = {k: params[k].grad.cpu().numpy().astype(np.float64) for k in TRAIN_KEYS}
    after = {k: params[k].detach().cpu().numpy().astype(np.float64) for k in TRAIN_KEYS}
    ex = {k: M.mgs_frame_export(rast.ctx, trainer.frame, k) for k in ("records", "radius", "depth")}
    torch.cuda.synchronize()
    # masks: the training sampler at step 0 of the counter, bit for bit
    m, y = oracle.sample_masks(tr["mask_scores"], tau, seed, 0)
    assert np.array_equal(rast.last_masks.cpu().numpy().astype(np.float64), m)
    assert float(rec.mask_loss) == pytest.approx(m.mean() ** 2, rel=1e-6)
    # the oracle on the GPU's own records (stage protocol), with the L1
    # gradient of the GPU's image (sign decided on the same FP32 values)
    oi = U.oracle_inputs_from_rec(ex["records"].view(-1, 12))
    rad = ex["radius"].cpu().numpy().astype(np.float64)
    dbits = U.u32(ex["depth"])
    ol = oracle.build_lists([128], [128], n, oi["mean2d"], rad, dbits, (rad > 0).astype(np.uint8), ost)
    of = oracle.render_fwd([128], [128], n, oi["mean2d"], oi["conic"], oi["opacity"], oi["color"], m, ol, ost)
    ok = of.flags == 0
    assert ok.mean() > 0.995
    scale = max(np.abs(of.image).max(), 1.0)
    assert np.abs(img - of.image)[np.tile(ok, 3)].max() <= 1e-5 * scale
    loss, dl = oracle.l1_loss(img, target)
    assert float(rec.l1) == pytest.approx(loss, rel=1e-6)
    ob = oracle.render_bwd([128], [128], n, oi["mean2d"], oi["conic"], oi["opacity"], oi["color"], m, ol, dl, ost)
    og = oracle.project_bwd(tr, [crop], ost, ob.d_mean2d, ob.d_conic, ob.d_opacity, ob.d_color)
    d_scores, _ = oracle.mask_grad(ob.d_mask, m, y, tau, lam)
    excl = ob.touched_flagged.astype(bool)
    want = {"means": og.means, "log_scales": og.log_scales, "quats": og.quats, "opacity_logits": og.opacity_logits,
            "sh": og.sh, "mask_scores": d_scores}
    for k in TRAIN_KEYS:
        U.assert_grad_close(g[k], want[k], excl, name=k)
    # Adam (first step): the update of the GPU's own gradients is the
    # oracle's Adam to FP32 rounding; where the oracle's gradient exceeds the
    # gradient tolerance the signs agree and so do the updates
    from paper_2412_20522_amd.train import ADAM_BETAS, ADAM_EPS, DEFAULT_LRS
    for k in TRAIN_KEYS:
        lr = DEFAULT_LRS[k]
        p1 = before[k].copy()
        oracle.adam(p1, g[k].copy(), np.zeros_like(p1), np.zeros_like(p1), lr, ADAM_BETAS[0], ADAM_BETAS[1],
                    ADAM_EPS, 1)
        assert np.all(np.abs(after[k] - p1) <= 2e-6 * (np.abs(p1) + lr)), k
        p2 = before[k].copy()
        oracle.adam(p2, want[k].copy(), np.zeros_like(p2), np.zeros_like(p2), lr, ADAM_BETAS[0], ADAM_BETAS[1],
                    ADAM_EPS, 1)
        o = want[k]
        # the first Adam step moves each parameter by about lr sign(g): where
        # the GPU's gradient and the oracle's have the same sign (or are both
        # 0) the updates agree; the others are gradients within the tolerance
        # of 0 (asserted above; for the scores, where the rendering gradient
        # and the L_m term nearly cancel), a small share of the non-zero ones
        agree = np.sign(g[k]) == np.sign(o)
        nz = (g[k] != 0) | (o != 0)
        assert (~agree).sum() <= max(2, 1e-2 * nz.sum()), (k, int((~agree).sum()), int(nz.sum()))
        # (gradients within a few decades of eps = 1e-15 move by lr g / (|g| + eps),
        # which depends on |g| itself: those are left to the check above)
        sure = agree & ((np.abs(o) > 1e-9) | (o == 0))
        assert np.all(np.abs(after[k] - p2)[sure] <= 2e-6 * (np.abs(p2) + lr)[sure]), k
    trainer.close()


def test_captured_training_steps_advance_counter_and_match_eager():
    """Steps replayed from per-batch graphs equal eager steps from the same
    state (the device counter gives each replay fresh masks and the next
    Adam step)."""
    from paper_2412_20522_amd.raster import Rasterizer
    from paper_2412_20522_amd.train import Trainer
    s = _scene_views()
    cams = s["cameras"]
    batches = [[cams[0], cams[1]], [cams[2]]]
    targets = [_targets(b, 10 + i) for i, b in enumerate(batches)]

    def make():
        rast = Rasterizer(0, sh_degree=2, bg=(0.1, 0.2, 0.3), persistent=1)
        params = {k: torch.from_numpy(np.ascontiguousarray(s[k], np.float32)).cuda() for k in TRAIN_KEYS}
        return Trainer(rast, params, batches, targets, tau=0.5, seed=5, lambda_m=0.2)

    eager = make()
    eager.reserve(1.5)
    for _ in range(6):
        eager.step()
    torch.cuda.synchronize()
    graphed = make()
    graphed.reserve(1.5)
    graphed.warmup(2)
    graphed.capture()
    for _ in range(4):
        graphed.step()
    torch.cuda.synchronize()
    graphed.check()
    assert int(graphed.counter.item()) == 6 == int(eager.counter.item())
    for k in TRAIN_KEYS:
        a = graphed.params[k].detach().cpu().numpy()
        b = eager.params[k].detach().cpu().numpy()
        assert U.rel_err(a, b) <= 1e-4, k
    eager.close()
    graphed.close()
