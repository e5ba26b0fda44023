"""Mask-application variants of the ablations (Sec. 4.3) through the C ABI,
against the oracle: mask x opacity (Table 7) for the whole path, and the
deterministic straight-through masks (Table 6).  Also the mechanism the
paper gives for the first one's "death spiral": under mask x opacity an
unsampled Gaussian gets no gradient at all, under masked rasterization it
gets dL/dM (Eq. 6) while the images agree."""
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


def _settings(deg, bg, mode, wide, cull):
    return dict(sh_degree=deg, bg=bg, tile_w=16, tile_h=16, batch_depth=128, fwd_ppt=4, bwd_ppt=4, persistent=1,
                exact_mode=0, wide_tiles=wide, tile_cull=cull, stats=0, mask_mode=mode)


def _run(rast, s, cams, masks, dl, **st):
    rast.set(**st)
    dev = U.to_device(s, masks)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    frame = rast.acquire_frame()
    img = rast.forward(frame, params, dev["masks"], cams).clone()
    g = rast.backward(frame, params, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    rast.release_frame(frame)
    rast.set(mask_mode=0)
    return img.cpu().numpy().astype(np.float64), g


def _scene(kind):
    if kind == "tiny":
        return scenegen.tiny_scene(), (0.0, 0.0, 0.0)
    if kind == "ragged":
        return scenegen.small_scene(3000, 150, 90, seed=301, sh_degree=3, log_scale_mean=-2.6), (0.2, 0.4, 0.6)
    return scenegen.small_scene(4000, 120, 96, seed=302, sh_degree=2, log_scale_mean=-2.5, n_views=3), (0.5, 0.1, 0.3)


@pytest.mark.parametrize("kind", ["tiny", "ragged", "multiview"])
@pytest.mark.parametrize("wide,cull", [(-1, 0), (8, 1), (1, 1)])
@pytest.mark.parametrize("fractional", [False, True])
def test_opacity_mode_matches_oracle(rast, kind, wide, cull, fractional):
    s, bg = _scene(kind)
    cams = s["cameras"]
    n = s["means"].shape[0]
    P = sum(c["width"] * c["height"] for c in cams)
    rng = np.random.default_rng(17)
    masks = rng.uniform(0.0, 1.0, n).astype(np.float32) if fractional else s["masks"].astype(np.float32)
    dl = rng.normal(size=3 * P).astype(np.float32)
    img, g = _run(rast, s, cams, masks, dl, **_settings(s["sh_degree"], bg, 1, wide, cull))
    ost = oracle.RasterSettings(sh_degree=s["sh_degree"], bg=bg)
    op = oracle.run_pipeline(s, cams, masks.astype(np.float64), ost, dl_dimage=dl.astype(np.float64),
                             mask_mode="opacity")
    assert U.rel_err(img, op.fwd.image) <= 2e-4
    assert np.abs(img - op.fwd.image).max() <= 2e-2
    for name, a, b in [("means", g.means, op.grads.means), ("log_scales", g.log_scales, op.grads.log_scales),
                       ("quats", g.quats, op.grads.quats),
                       ("opacity_logits", g.opacity_logits, op.grads.opacity_logits),
                       ("sh", g.sh, op.grads.sh), ("masks", g.masks, op.bwd.d_mask)]:
        e = U.rel_err(a.cpu().numpy(), b)
        assert e <= 2e-3, (name, e)
    if not fractional:
        assert torch.all(g.masks[torch.from_numpy(masks == 0).cuda()] == 0).item()


@pytest.mark.parametrize("cull", [0, 1])
def test_unsampled_gaussians_get_no_gradient_under_mask_x_opacity(rast, cull):
    s, bg = _scene("ragged")
    cams = s["cameras"]
    P = sum(c["width"] * c["height"] for c in cams)
    masks = s["masks"].astype(np.float32)
    dl = np.random.default_rng(18).normal(size=3 * P).astype(np.float32)
    img0, g0 = _run(rast, s, cams, masks, dl, **_settings(3, bg, 0, 8, cull))
    img1, g1 = _run(rast, s, cams, masks, dl, **_settings(3, bg, 1, 8, cull))
    np.testing.assert_allclose(img1, img0, rtol=0, atol=1e-6)
    off = torch.from_numpy(masks == 0).cuda()
    assert torch.all(g1.masks[off] == 0).item()
    assert torch.count_nonzero(g0.masks[off]).item() >= 0.3 * int(off.sum())
    for name in U.PARAM_KEYS:
        a, b = getattr(g0, name), getattr(g1, name)
        assert torch.count_nonzero(a[off]).item() == 0 and torch.count_nonzero(b[off]).item() == 0, name
        assert U.rel_err(b.cpu().numpy(), a.cpu().numpy().astype(np.float64)) <= 1e-4, name


@pytest.mark.parametrize("n", [0, 1, 100_003])
@pytest.mark.parametrize("thr", [0.01, 0.5])
def test_threshold_masks_match_oracle(n, thr):
    ctx = U.M().mgs_create(0)
    rng = np.random.default_rng(n + 1)
    scores = (rng.normal(size=(n, 2)) * 3.0).astype(np.float32)
    m = torch.full((max(n, 1),), -1.0, device="cuda")
    y = torch.full((max(n, 1),), -1.0, device="cuda")
    U.M().mgs_threshold_masks(ctx, torch.from_numpy(scores).cuda().reshape(n, 2), thr, m[:n], y[:n])
    torch.cuda.synchronize()
    om, oy = oracle.threshold_masks(scores.astype(np.float64), thr)
    assert np.array_equal(m[:n].cpu().numpy(), om.astype(np.float32))
    if n:
        assert np.abs(y[:n].cpu().numpy() - oy).max() <= 1e-7


def test_invalid_mask_mode_is_rejected(rast):
    s, bg = _scene("tiny")
    rast.set(mask_mode=2)
    dev = U.to_device(s, None)
    frame = rast.acquire_frame()
    try:
        with pytest.raises(U.M().MaskGSError):
            rast.forward(frame, {k: dev[k] for k in U.PARAM_KEYS}, dev["masks"], s["cameras"])
    finally:
        rast.release_frame(frame)
        rast.set(mask_mode=0)


def test_opacity_mode_exact_mode_matches_oracle(rast):
    """No alpha filter, stop or Q cut: mask x opacity against the oracle with
    fractional masks, where unsampled Gaussians do receive gradients."""
    s, bg = _scene("tiny")
    cams = s["cameras"]
    n = s["means"].shape[0]
    P = sum(c["width"] * c["height"] for c in cams)
    rng = np.random.default_rng(19)
    masks = rng.uniform(0.0, 1.0, n).astype(np.float32)
    masks[::5] = 0.0
    dl = rng.normal(size=3 * P).astype(np.float32)
    st = _settings(s["sh_degree"], bg, 1, -1, 0)
    st["exact_mode"] = 1
    img, g = _run(rast, s, cams, masks, dl, **st)
    ost = oracle.RasterSettings(sh_degree=s["sh_degree"], bg=bg, exact_mode=True)
    op = oracle.run_pipeline(s, cams, masks.astype(np.float64), ost, dl_dimage=dl.astype(np.float64),
                             mask_mode="opacity")
    assert U.rel_err(img, op.fwd.image) <= 2e-4
    for name, a, b in [("means", g.means, op.grads.means), ("opacity_logits", g.opacity_logits,
                                                             op.grads.opacity_logits),
                       ("sh", g.sh, op.grads.sh), ("masks", g.masks, op.bwd.d_mask)]:
        e = U.rel_err(a.cpu().numpy(), b)
        assert e <= 2e-3, (name, e)
    # without the filter an unsampled Gaussian's alpha is 0, not filtered out
    assert np.count_nonzero(op.bwd.d_mask[masks == 0]) > 0
