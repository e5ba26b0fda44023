"""Degenerate and maximum sizes of the whole path: no Gaussians, no visible
Gaussian, the largest number of views (16, ragged sizes down to one pixel)
against the oracle, and more views than allowed refused on the host."""
import ctypes as C

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
    return Rasterizer(0, sh_degree=1, bg=(0.25, 0.5, 0.75), persistent=1, tile_cull=1, wide_tiles=8)


def _bg_image(cams, bg):
    return np.concatenate([np.repeat(np.float32(bg).astype(np.float64)[:, None], c["width"] * c["height"], axis=1)
                           .reshape(-1) for c in cams])


def _cut(s, idx):
    return {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == s["means"].shape[:1] else v)
            for k, v in s.items()}


def test_no_gaussians_renders_the_background(rast):
    s = _cut(scenegen.small_scene(10, 40, 30, seed=501, sh_degree=1), slice(0, 0))
    cams = s["cameras"] + [scenegen.orbit_camera(4.0, 60.0, 0.0, 17, 9)]
    dev = U.to_device(s)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    P = sum(c["width"] * c["height"] for c in cams)
    frame = rast.acquire_frame()
    tfin = torch.empty(P, device="cuda")
    img = rast.forward(frame, params, dev["masks"], cams, t_final=tfin).clone()
    g = rast.backward(frame, params, torch.ones(3 * P, device="cuda"))
    img2, isum, imax = rast.forward_importance(frame, params, dev["masks"], cams)
    torch.cuda.synchronize()
    rast.release_frame(frame)
    assert np.array_equal(img.cpu().numpy().astype(np.float64), _bg_image(cams, (0.25, 0.5, 0.75)))
    assert torch.equal(img, img2) and torch.all(tfin == 1.0).item()
    assert g.means.numel() == 0 and g.masks.numel() == 0 and isum.numel() == 0


def test_no_visible_gaussian_renders_the_background(rast):
    """Every Gaussian behind the camera: no record, no list entry; the
    background, transmittance 1 and zero gradients everywhere."""
    s = scenegen.small_scene(500, 40, 30, seed=502, sh_degree=1)
    s["means"] = s["means"].copy()
    s["means"][:, 2] = -np.abs(s["means"][:, 2]) - 10.0  # the camera looks down +z from the origin side
    cam = scenegen.camera_from_pose(np.eye(3), np.zeros(3), 40, 30)
    dev = U.to_device(s)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    frame = rast.acquire_frame()
    img = rast.forward(frame, params, dev["masks"], [cam]).clone()
    g = rast.backward(frame, params, torch.ones(3 * 40 * 30, device="cuda"))
    stats = rast.stats(frame)
    torch.cuda.synchronize()
    rast.release_frame(frame)
    assert stats["n_instances"] == 0
    assert np.array_equal(img.cpu().numpy().astype(np.float64), _bg_image([cam], (0.25, 0.5, 0.75)))
    for name in U.PARAM_KEYS + ("masks",):
        assert torch.count_nonzero(getattr(g, name)).item() == 0, name


def test_sixteen_ragged_views_match_oracle(rast):
    """The largest view count, with views from 1x1 to 150x90 pixels."""
    s = scenegen.small_scene(2500, 64, 48, seed=503, sh_degree=1, log_scale_mean=-2.4)
    sizes = [(64, 48), (1, 1), (1, 33), (33, 1), (17, 9), (150, 90), (16, 16), (31, 47),
             (2, 2), (80, 15), (15, 80), (48, 64), (100, 3), (7, 7), (65, 33), (40, 40)]
    cams = [scenegen.orbit_camera(4.0, 22.5 * k, 10.0 * ((k % 3) - 1), w, h) for k, (w, h) in enumerate(sizes)]
    assert len(cams) == 16
    P = sum(w * h for w, h in sizes)
    dl = np.random.default_rng(9).normal(size=3 * P).astype(np.float32)
    dev = U.to_device(s)
    params = {k: dev[k] for k in U.PARAM_KEYS}
    frame = rast.acquire_frame()
    img = rast.forward(frame, params, dev["masks"], cams).clone()
    g = rast.backward(frame, params, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    rast.release_frame(frame)
    op = oracle.run_pipeline(s, cams, s["masks"].astype(np.float64),
                             oracle.RasterSettings(sh_degree=1, bg=(0.25, 0.5, 0.75)), dl_dimage=dl.astype(np.float64))
    gi = img.cpu().numpy().astype(np.float64)
    assert U.rel_err(gi, op.fwd.image) <= 2e-4
    assert np.abs(gi - op.fwd.image).max() <= 2e-2
    for name, a, b in [("means", g.means, op.grads.means), ("log_scales", g.log_scales, op.grads.log_scales),
                       ("opacity_logits", g.opacity_logits, op.grads.opacity_logits), ("sh", g.sh, op.grads.sh),
                       ("masks", g.masks, op.bwd.d_mask)]:
        e = U.rel_err(a.cpu().numpy(), b)
        assert e <= 2e-3, (name, e)


def test_seventeen_views_are_refused(rast):
    s = scenegen.small_scene(100, 16, 16, seed=504, sh_degree=1)
    cams = [scenegen.orbit_camera(4.0, 20.0 * k, 0.0, 16, 16) for k in range(17)]
    dev = U.to_device(s)
    M = U.M()
    frame = rast.acquire_frame()
    try:
        # the binding refuses them before the call ...
        with pytest.raises(ValueError):
            rast.forward(frame, {k: dev[k] for k in U.PARAM_KEYS}, dev["masks"], cams)
        # ... and so does the library, through the C ABI, on the host
        ca = (M.mgs_camera * 17)(*[M.camera_struct(c) for c in cams])
        g = M.gaussians_struct(*(dev[k] for k in U.PARAM_KEYS), dev["masks"])
        img = torch.empty(3 * 16 * 16 * 17, device="cuda")
        rc = M.lib().mgs_forward(frame, M._stream(None), C.byref(g), ca, 17, C.byref(rast.settings),
                                 C.c_void_p(img.data_ptr()), None)
        assert M.STATUS[rc] == "MGS_ERR_INVALID_ARG"
    finally:
        rast.release_frame(frame)
