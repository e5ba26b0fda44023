"""End-to-end parity of the whole HIP path (mgs_forward / mgs_backward and the
autograd Function) with the FP64 oracle, plus the method's special cases and
invariants on the GPU."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    from paper_2412_20522_amd.raster import Rasterizer
    return Rasterizer(0)


def _params(dev):
    return {k: dev[k] for k in U.PARAM_KEYS}


def _render(rast, scene, cams, masks=None, dl=None, **settings):
    rast.set(**settings)
    dev = U.to_device(scene, masks)
    frame = rast.acquire_frame()
    P = sum(c["width"] * c["height"] for c in cams)
    tfin = torch.empty(P, device="cuda")
    img = rast.forward(frame, _params(dev), dev["masks"], cams, t_final=tfin)
    out = None
    if dl is not None:
        out = rast.backward(frame, _params(dev), torch.from_numpy(np.asarray(dl, np.float32)).cuda())
    torch.cuda.synchronize()
    stats = rast.stats(frame)
    evals = rast.count_evals(frame)
    rast.release_frame(frame)
    return img.cpu().numpy().astype(np.float64), tfin.cpu().numpy(), out, stats, evals


def _defaults(deg, bg=(0.0, 0.0, 0.0), **kw):
    base = dict(tile_w=16, tile_h=16, batch_depth=256, fwd_ppt=1, bwd_ppt=4, persistent=0, exact_mode=0,
                wide_tiles=0, tile_cull=1, stats=1)
    base.update(kw)
    return dict(sh_degree=deg, bg=bg, **base)


@pytest.mark.parametrize("kind", ["tiny", "ragged"])
@pytest.mark.parametrize("wide", [-1, 0, 1])
@pytest.mark.parametrize("cull", [0, 1])
def test_full_path_matches_oracle(rast, kind, wide, cull):
    """Whole path against the oracle with plain binning (wide = -1), the
    automatic wide-list threshold (0) and nearly every record in the wide
    lists (1); with the lists of Sec. 3.1 exactly (cull = 0) and with narrow
    instances only for tiles a record can reach (cull = 1)."""
    if kind == "tiny":
        s = scenegen.tiny_scene()
        bg = (0.0, 0.0, 0.0)
    else:
        s = scenegen.small_scene(3000, 150, 90, seed=201, sh_degree=3, log_scale_mean=-2.6)
        bg = (0.2, 0.4, 0.6)
    cams = s["cameras"]
    P = sum(c["width"] * c["height"] for c in cams)
    rng = np.random.default_rng(5)
    dl = rng.normal(size=3 * P).astype(np.float32)
    img, tfin, g, stats, evals = _render(rast, s, cams, dl=dl, **_defaults(s["sh_degree"], bg, wide_tiles=wide,
                                                                          tile_cull=cull))
    ost = oracle.RasterSettings(sh_degree=s["sh_degree"], bg=bg)
    op = oracle.run_pipeline(s, cams, s["masks"].astype(np.float64), ost, dl_dimage=dl.astype(np.float64))
    # images: FP32 pixel coordinates limit agreement with the FP64 projection
    assert U.rel_err(img, op.fwd.image) <= 2e-4
    assert np.abs(img - op.fwd.image).max() <= 2e-2
    if wide < 0:
        assert stats["n_wide"] == 0
    if wide < 0 and not cull:
        assert stats["n_instances"] == pytest.approx(op.lists.keys.size, rel=1e-3)
    else:
        assert stats["n_instances"] <= op.lists.keys.size * (1 + 1e-3)
    if wide == 1:
        assert stats["n_wide"] > 0
    if not cull:
        assert evals["examined"] == pytest.approx(int(op.fwd.examined.sum()), rel=1e-3)
    else:
        assert evals["examined"] <= int(op.fwd.examined.sum()) * (1 + 1e-3)
    assert evals["blended"] == pytest.approx(int(op.fwd.n_blend.sum()), rel=1e-3)
    assert 0 < evals["blended_masked"] < evals["blended"]
    assert evals["examined"] >= evals["bwd_examined"] >= evals["blended"]
    # the per-tile test only drops entries that cannot reach a pixel of the tile
    assert evals["examined"] >= evals["evaluated"] >= evals["bwd_evaluated"] >= evals["blended"]
    for name, a, b in [("means", g.means, op.grads.means), ("log_scales", g.log_scales, op.grads.log_scales),
                       ("quats", g.quats, op.grads.quats), ("opacity_logits", g.opacity_logits,
                                                             op.grads.opacity_logits),
                       ("sh", g.sh, op.grads.sh), ("masks", g.masks, op.bwd.d_mask)]:
        e = U.rel_err(a.cpu().numpy(), b)
        assert e <= 2e-3, (name, e)


def test_zero_masks_render_background_exactly(rast):
    s = scenegen.small_scene(2000, 120, 80, seed=202, sh_degree=2, log_scale_mean=-2.5)
    bg = (0.25, 0.5, 0.75)
    P = 120 * 80
    dl = np.random.default_rng(6).normal(size=3 * P).astype(np.float32)
    img, tfin, g, _, _ = _render(rast, s, s["cameras"], masks=np.zeros(2000, np.float32), dl=dl,
                                 **_defaults(2, bg))
    want = np.repeat(np.float32(bg).astype(np.float64)[:, None], P, axis=1).reshape(-1)
    assert np.array_equal(img, want)
    assert np.all(tfin == 1.0)
    for t in (g.means, g.log_scales, g.quats, g.opacity_logits, g.sh):
        assert torch.count_nonzero(t).item() == 0
    # and the mask gradient is the closed form sum_px alpha <w, c - bg> (compare with the oracle)
    ost = oracle.RasterSettings(sh_degree=2, bg=bg)
    op = oracle.run_pipeline(s, s["cameras"], np.zeros(2000), ost, dl_dimage=dl.astype(np.float64))
    assert U.rel_err(g.masks.cpu().numpy(), op.bwd.d_mask) <= 2e-3


def test_forward_is_deterministic_and_backward_reproducible(rast):
    s = scenegen.small_scene(4000, 160, 120, seed=203, sh_degree=3, log_scale_mean=-2.5)
    dl = np.random.default_rng(8).normal(size=3 * 160 * 120).astype(np.float32)
    a = _render(rast, s, s["cameras"], dl=dl, **_defaults(3))
    b = _render(rast, s, s["cameras"], dl=dl, **_defaults(3))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip((a[2].means, a[2].masks, a[2].sh), (b[2].means, b[2].masks, b[2].sh)):
        assert U.rel_err(x.cpu().numpy(), y.cpu().numpy()) <= 1e-5


def test_tile_culling_changes_nothing_but_the_lists(rast):
    """Dropping narrow instances whose record cannot reach a pixel of the
    tile leaves images and final transmittance bit for bit and gradients to
    FP64-atomics reordering, with fewer instances."""
    s = scenegen.small_scene(4000, 140, 100, seed=206, sh_degree=2, log_scale_mean=-2.0, n_views=2)
    s["cameras"][1] = scenegen.orbit_camera(4.0, 60.0, 10.0, 96, 64)
    P = sum(c["width"] * c["height"] for c in s["cameras"])
    dl = np.random.default_rng(11).normal(size=3 * P).astype(np.float32)
    out = {}
    for cull in (0, 1):
        out[cull] = _render(rast, s, s["cameras"], dl=dl, **_defaults(2, (0.2, 0.3, 0.4), tile_cull=cull,
                                                                     persistent=1))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert out[1][3]["n_instances"] < out[0][3]["n_instances"]
    assert out[1][4]["blended"] == out[0][4]["blended"]
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh", "masks"):
        a = getattr(out[1][2], name).cpu().numpy()
        b = getattr(out[0][2], name).cpu().numpy()
        assert U.rel_err(a, b) <= 1e-5, name


def test_tile_shape_and_batch_invariance(rast):
    s = scenegen.small_scene(3000, 130, 100, seed=204, sh_degree=1, log_scale_mean=-2.4)
    ref = None
    for tw, th, fp, bp, bd in [(16, 16, 1, 4, 256), (8, 8, 1, 1, 32), (16, 8, 2, 2, 64), (32, 8, 4, 4, 128),
                               (16, 16, 4, 1, 64)]:
        img, tfin, _, _, _ = _render(rast, s, s["cameras"], **_defaults(1, tile_w=tw, tile_h=th, fwd_ppt=fp,
                                                                         bwd_ppt=bp, batch_depth=bd))
        if ref is None:
            ref = img
        else:
            assert np.abs(img - ref).max() <= 1e-6


def test_multiview_batch_equals_single_views_and_persistent(rast):
    s = scenegen.small_scene(3000, 90, 70, seed=205, sh_degree=2, log_scale_mean=-2.5, n_views=4)
    cams = s["cameras"]
    cams[1] = scenegen.orbit_camera(4.0, 30.0, 5.0, 64, 96)
    cams[3] = scenegen.orbit_camera(4.0, -40.0, -5.0, 33, 47)
    P = sum(c["width"] * c["height"] for c in cams)
    dl = np.random.default_rng(9).normal(size=3 * P).astype(np.float32)
    full, _, gfull, _, _ = _render(rast, s, cams, dl=dl, **_defaults(2))
    pers, _, gpers, _, _ = _render(rast, s, cams, dl=dl, **_defaults(2, persistent=1))
    assert np.array_equal(full, pers)
    assert U.rel_err(gpers.means.cpu().numpy(), gfull.means.cpu().numpy()) <= 1e-5
    off = 0
    gsum = np.zeros_like(gfull.means.cpu().numpy(), dtype=np.float64)
    msum = np.zeros(3000)
    for c in cams:
        p = c["width"] * c["height"]
        one, _, g1, _, _ = _render(rast, s, [c], dl=dl[3 * off:3 * (off + p)], **_defaults(2))
        assert np.array_equal(one, full[3 * off:3 * (off + p)])
        gsum += g1.means.cpu().numpy()
        msum += g1.masks.cpu().numpy()
        off += p
    assert U.rel_err(gfull.means.cpu().numpy(), gsum) <= 1e-5
    assert U.rel_err(gfull.masks.cpu().numpy(), msum) <= 1e-5


def test_autograd_function_straight_through(rast):
    from paper_2412_20522_amd.raster import masked_rasterize
    s = scenegen.small_scene(2000, 96, 64, seed=206, sh_degree=1, log_scale_mean=-2.4)
    rast.set(**_defaults(1))
    dev = U.to_device(s)
    params = {k: dev[k].clone().requires_grad_(True) for k in U.PARAM_KEYS}
    scores = dev["mask_scores"].clone().requires_grad_(True)
    target = torch.rand(3 * 96 * 64, device="cuda")
    images, mask_loss = masked_rasterize(params, scores, rast, s["cameras"], tau=0.5, seed=11, step=3)
    loss = (images - target).abs().mean() + 0.1 * mask_loss
    loss.backward()
    m_hard = rast.last_masks.cpu().numpy().astype(np.float64)
    om, oy = oracle.sample_masks(s["mask_scores"], 0.5, 11, 3)
    assert np.array_equal(m_hard, om)
    # the score gradient is the straight-through chain of dL/dM and the mask loss
    ost = oracle.RasterSettings(sh_degree=1)
    dl = np.sign(images.detach().cpu().numpy().astype(np.float64) - target.cpu().numpy()) / target.numel()
    op = oracle.run_pipeline(s, s["cameras"], om, ost, dl_dimage=dl)
    od, _ = oracle.mask_grad(op.bwd.d_mask, om, oy, 0.5, 0.1)
    assert U.rel_err(scores.grad.cpu().numpy(), od) <= 2e-3
    assert U.rel_err(params["means"].grad.cpu().numpy(), op.grads.means) <= 2e-3
    assert abs(mask_loss.item() - om.mean() ** 2) <= 1e-6


@pytest.mark.parametrize("n_views", [1, 3])
def test_backward_returns_per_record_2d_gradients(rast, n_views):
    """The optional per-record output of mgs_backward against the oracle's
    per-record gradients (conic converted to the stored basis), and the
    parameter gradients unchanged by asking for it."""
    s = scenegen.small_scene(3000, 120, 96, seed=211, sh_degree=2, log_scale_mean=-2.5, n_views=n_views)
    bg = (0.3, 0.1, 0.2)
    cams = s["cameras"]
    n = s["means"].shape[0]
    P = sum(c["width"] * c["height"] for c in cams)
    dl = np.random.default_rng(12).normal(size=3 * P).astype(np.float32)
    rast.set(**_defaults(2, bg))
    dev = U.to_device(s)
    frame = rast.acquire_frame()
    rast.forward(frame, _params(dev), dev["masks"], cams)
    recs = torch.full((n_views * n, 9), 7.0, device="cuda")
    g = rast.backward(frame, _params(dev), torch.from_numpy(dl).cuda(), records=recs)
    g_plain = rast.backward(frame, _params(dev), torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    rast.release_frame(frame)
    ost = oracle.RasterSettings(sh_degree=2, bg=bg)
    op = oracle.run_pipeline(s, cams, s["masks"].astype(np.float64), ost, dl_dimage=dl.astype(np.float64))
    got = recs.cpu().numpy().astype(np.float64)
    m2d, con, _, _, _, _, valid = oracle.stack_projected(op.proj)
    assert np.all(got[~valid.astype(bool)] == 0.0)
    want_conic = U.dstable_from_dabc(con[:, 0], con[:, 1] / np.where(con[:, 0] != 0, con[:, 0], 1.0), op.bwd.d_conic)
    for name, a, b in [("mean2d", got[:, 0:2], op.bwd.d_mean2d), ("conic", got[:, 2:5], want_conic),
                       ("opacity", got[:, 5], op.bwd.d_opacity), ("color", got[:, 6:9], op.bwd.d_color)]:
        e = U.rel_err(a, b)
        assert e <= 2e-3, (name, e)
    for name in U.PARAM_KEYS + ("masks",):
        a, b = getattr(g, name).cpu().numpy(), getattr(g_plain, name).cpu().numpy()
        assert U.rel_err(a, b.astype(np.float64)) <= 1e-6, name
