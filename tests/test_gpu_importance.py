"""Importance by-products of the forward (mgs_forward_importance) against the
oracle: per Gaussian, the sum and the maximum over every pixel of every view
of its blending weight M alpha T.  Also: the importance forward renders the
same images as mgs_forward, leaves a frame the backward accepts with the
same gradients, and obeys the telescoping identity (weights plus final
transmittance add up to 1 per pixel) at full size."""
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


def _scene(kind):
    if kind == "tiny":
        return scenegen.tiny_scene(), (0.0, 0.0, 0.0)
    if kind == "ragged":
        return scenegen.small_scene(3000, 150, 90, seed=401, sh_degree=3, log_scale_mean=-2.6), (0.2, 0.4, 0.6)
    return scenegen.small_scene(4000, 120, 96, seed=402, sh_degree=2, log_scale_mean=-2.5, n_views=3), (0.5, 0.1, 0.3)


@pytest.mark.parametrize("kind", ["tiny", "ragged", "multiview"])
@pytest.mark.parametrize("wide,cull,ppt", [(-1, 0, 1), (8, 1, 4), (1, 1, 2)])
def test_importance_matches_oracle(rast, kind, wide, cull, ppt):
    s, bg = _scene(kind)
    cams = s["cameras"]
    rast.set(sh_degree=s["sh_degree"], bg=bg, tile_w=16, tile_h=16, batch_depth=128, fwd_ppt=ppt, bwd_ppt=4,
             persistent=1, exact_mode=0, wide_tiles=wide, tile_cull=cull, stats=1, mask_mode=0)
    dev = U.to_device(s)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    frame = rast.acquire_frame()
    img, isum, imax = rast.forward_importance(frame, params, dev["masks"], cams)
    img, isum, imax = img.clone(), isum.clone(), imax.clone()
    ref = rast.forward(frame, params, dev["masks"], cams).clone()
    torch.cuda.synchronize()
    rast.release_frame(frame)
    assert torch.equal(img, ref)
    ost = oracle.RasterSettings(sh_degree=s["sh_degree"], bg=bg)
    os_, om = oracle.scene_importance(s, cams, s["masks"].astype(np.float64), ost)
    gs, gm = isum.cpu().numpy(), imax.cpu().numpy()
    assert U.rel_err(gs, os_) <= 1e-3
    assert U.rel_err(gm, om) <= 1e-3
    off = s["masks"] == 0
    assert np.all(gs[off] == 0.0) and np.all(gm[off] == 0.0)
    assert np.all(gm <= gs * (1 + 1e-6) + 1e-30)


def test_backward_after_importance_forward(rast):
    s, bg = _scene("ragged")
    cams = s["cameras"]
    rast.set(sh_degree=3, bg=bg, tile_w=16, tile_h=16, batch_depth=128, fwd_ppt=4, bwd_ppt=4, persistent=1,
             exact_mode=0, wide_tiles=8, tile_cull=1, stats=0, mask_mode=0)
    dev = U.to_device(s)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    P = sum(c["width"] * c["height"] for c in cams)
    dl = torch.from_numpy(np.random.default_rng(3).normal(size=3 * P).astype(np.float32)).cuda()
    fa, fb = rast.acquire_frame(), rast.acquire_frame()
    rast.forward(fa, params, dev["masks"], cams)
    ga = rast.backward(fa, params, dl)
    rast.forward_importance(fb, params, dev["masks"], cams)
    gb = rast.backward(fb, params, dl)
    torch.cuda.synchronize()
    for name in U.PARAM_KEYS + ("masks",):
        a, b = getattr(ga, name).cpu().numpy(), getattr(gb, name).cpu().numpy()
        assert U.rel_err(b, a.astype(np.float64)) <= 1e-6, name
    rast.release_frame(fa)
    rast.release_frame(fb)


def test_importance_telescopes_at_full_size(rast):
    """Batched workload (1M Gaussians, 8 views): the weights of all Gaussians
    add up to the number of pixels minus the total final transmittance."""
    s = scenegen.batched_scene()
    cams = s["cameras"]
    rast.set(sh_degree=3, bg=(0.0, 0.0, 0.0), tile_w=16, tile_h=16, batch_depth=128, fwd_ppt=4, bwd_ppt=4,
             persistent=1, exact_mode=0, wide_tiles=8, tile_cull=1, stats=0, mask_mode=0)
    dev = U.to_device(s, np.ones(s["means"].shape[0], np.float32))
    params = {k: dev[k] for k in U.PARAM_KEYS}
    masks = dev["masks"]
    P = sum(c["width"] * c["height"] for c in cams)
    tfin = torch.empty(P, device="cuda")
    frame = rast.acquire_frame()
    g = U.M().gaussians_struct(*(params[k] for k in U.PARAM_KEYS), masks)
    img = torch.empty(3 * P, device="cuda")
    isum = torch.empty_like(masks)
    imax = torch.empty_like(masks)
    U.M().mgs_forward_importance(rast.ctx, frame, g, cams, rast.settings, img, isum, imax, t_final=tfin)
    torch.cuda.synchronize()
    rast.release_frame(frame)
    total = float(isum.double().sum())
    want = P - float(tfin.double().sum())
    assert abs(total - want) <= 1e-4 * P
    assert float(imax.max()) <= 0.99 + 1e-6
    # the scene is strongly occluded: a view blends about 1 % of the Gaussians
    assert int(torch.count_nonzero(isum)) > 20_000


def test_importance_matches_oracle_at_full_size(rast):
    """The 1M-Gaussian scene seen by its 640x480 view: every Gaussian's
    importance against the oracle."""
    s = scenegen.batched_scene()
    cam = s["cameras"][0]
    n = s["means"].shape[0]
    rast.set(sh_degree=3, bg=(0.0, 0.0, 0.0), tile_w=16, tile_h=16, batch_depth=128, fwd_ppt=4, bwd_ppt=4,
             persistent=1, exact_mode=0, wide_tiles=8, tile_cull=1, stats=0, mask_mode=0)
    dev = U.to_device(s, np.ones(n, np.float32))
    params = {k: dev[k] for k in U.PARAM_KEYS}
    frame = rast.acquire_frame()
    _, isum, imax = rast.forward_importance(frame, params, dev["masks"], [cam])
    torch.cuda.synchronize()
    rast.release_frame(frame)
    os_, om = oracle.scene_importance(s, [cam], np.ones(n), oracle.RasterSettings(sh_degree=3))
    gs, gm = isum.cpu().numpy(), imax.cpu().numpy()
    assert np.count_nonzero(os_) > 5000
    assert U.rel_err(gs, os_) <= 1e-3
    assert U.rel_err(gm, om) <= 1e-3
    # the Gaussians that matter most agree one by one
    top = np.argsort(-os_)[:1000]
    assert np.all(np.abs(gs[top] - os_[top]) <= 1e-3 * os_[top] + 1e-3)
