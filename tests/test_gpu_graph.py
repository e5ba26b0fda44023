"""Fixed workspace, captured training step (hipGraph through torch's graph
capture) and the autotuner of the batched multi-view path.

The captured step is replayed several times with eager work and
synchronisations between replays; every replay must reproduce the eager
step (images bit for bit, gradients to atomics reordering), and a forward
whose counts outgrow the fixed workspace must be reported, not crash."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _multiview_scene():
    s = scenegen.small_scene(3000, 96, 80, seed=301, sh_degree=2, log_scale_mean=-2.3, n_views=4)
    s["cameras"][1] = scenegen.orbit_camera(4.0, 30.0, 5.0, 64, 96)
    s["cameras"][2] = scenegen.orbit_camera(4.0, 150.0, 10.0, 120, 72)
    s["cameras"][3] = scenegen.orbit_camera(4.0, -40.0, -5.0, 33, 47)
    return s


@pytest.fixture(scope="module")
def rast():
    from paper_2412_20522_amd.raster import Rasterizer
    return Rasterizer(0, sh_degree=2, bg=(0.1, 0.2, 0.3), persistent=1)


def _setup(rast, s):
    from paper_2412_20522_amd.raster import PARAM_KEYS, Grads
    dev = U.to_device(s)
    params = {k: dev[k] for k in PARAM_KEYS}
    cams = s["cameras"]
    P = sum(c["width"] * c["height"] for c in cams)
    images = torch.empty(3 * P, device="cuda")
    dl = torch.from_numpy(np.random.default_rng(3).normal(size=3 * P).astype(np.float32)).cuda()
    grads = Grads(*(torch.empty_like(params[k]) for k in PARAM_KEYS), torch.empty(params["means"].shape[0],
                                                                                  device="cuda"))
    return dev, params, cams, images, dl, grads


def _step(rast, frame, params, masks, cams, images, dl, grads):
    rast.forward(frame, params, masks, cams, images=images)
    rast.backward(frame, params, dl, out=grads)


def _grads_np(g):
    return [x.detach().cpu().numpy().astype(np.float64) for x in (g.means, g.log_scales, g.quats,
                                                                  g.opacity_logits, g.sh, g.masks)]


def test_reserved_frame_and_graph_replays_match_eager(rast):
    s = _multiview_scene()
    dev, params, cams, images, dl, grads = _setup(rast, s)
    frame = rast.acquire_frame()
    try:
        _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.synchronize()
        ref_img = images.cpu().numpy().copy()
        ref_g = _grads_np(grads)
        st_plain = rast.stats(frame)
        rast.reserve(frame, 1.25)
        # eager step on the fixed workspace: no allocation, no synchronisation
        images.fill_(-1.0)
        _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        rast.check(frame)
        assert np.array_equal(images.cpu().numpy(), ref_img)
        for a, b in zip(_grads_np(grads), ref_g):
            assert U.rel_err(a, b) <= 1e-5
        assert rast.stats(frame)["n_instances"] == st_plain["n_instances"]
        # capture the step
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.synchronize()
        for rep in range(3):
            images.fill_(float(rep) - 5.0)
            for x in (grads.means, grads.masks):
                x.fill_(123.0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            rast.check(frame)
            assert np.array_equal(images.cpu().numpy(), ref_img), rep
            for a, b in zip(_grads_np(grads), ref_g):
                assert U.rel_err(a, b) <= 1e-5, rep
            # eager work between replays
            _ = (images * 2.0).sum().item()
        del graph
    finally:
        rast.reserve(frame, 0)
        rast.release_frame(frame)


def test_reserved_frame_reports_overflow_and_recovers(rast):
    from paper_2412_20522_amd import maskgs as M
    s = _multiview_scene()
    dev, params, cams, images, dl, grads = _setup(rast, s)
    frame = rast.acquire_frame()
    try:
        _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        rast.reserve(frame, 1.0)
        # larger splats: more instances and wide entries than reserved
        big = dict(params)
        big["log_scales"] = params["log_scales"] + 0.7
        rast.forward(frame, big, dev["masks"], cams, images=images)
        with pytest.raises(M.MaskGSError) as e:
            rast.check(frame)
        assert e.value.status == 3  # MGS_ERR_CAPACITY
        # more records than reserved: refused on the host
        s2 = scenegen.small_scene(4000, 96, 80, seed=302, sh_degree=2, n_views=4)
        dev2 = U.to_device(s2)
        p2 = {k: dev2[k] for k in params}
        with pytest.raises(M.MaskGSError):
            rast.forward(frame, p2, dev2["masks"], cams, images=images)
        # released: the plain path grows again and renders correctly
        rast.reserve(frame, 0)
        rast.forward(frame, big, dev["masks"], cams, images=images)
        rast.check(frame)
    finally:
        rast.reserve(frame, 0)
        rast.release_frame(frame)


def test_autotuner_returns_valid_settings_with_identical_images(rast):
    from paper_2412_20522_amd.raster import Rasterizer
    s = _multiview_scene()
    r = Rasterizer(0, sh_degree=2, bg=(0.1, 0.2, 0.3), persistent=1)
    dev, params, cams, images, dl, grads = _setup(r, s)
    frame = r.acquire_frame()
    try:
        _step(r, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.synchronize()
        ref = images.cpu().numpy().copy()
        best, ms = r.autotune(frame, params, dev["masks"], cams, dl)
        assert ms > 0
        assert (best["tile_w"], best["tile_h"]) in [(16, 16), (16, 8), (32, 8), (8, 8)]
        assert best["batch_depth"] in (32, 64, 128, 256)
        _step(r, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.synchronize()
        assert np.abs(images.cpu().numpy() - ref).max() <= 1e-6
    finally:
        r.release_frame(frame)


def test_graph_step_matches_oracle(rast):
    """A replay of the captured step against the FP64 oracle (images and the
    mask gradient), on one view with a non-black background."""
    s = scenegen.small_scene(2000, 100, 70, seed=303, sh_degree=2, log_scale_mean=-2.4)
    dev, params, cams, images, dl, grads = _setup(rast, s)
    frame = rast.acquire_frame()
    try:
        _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        rast.reserve(frame, 1.1)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            _step(rast, frame, params, dev["masks"], cams, images, dl, grads)
        images.zero_()
        graph.replay()
        torch.cuda.synchronize()
        rast.check(frame)
        ost = oracle.RasterSettings(sh_degree=2, bg=(0.1, 0.2, 0.3))
        op = oracle.run_pipeline(s, cams, s["masks"].astype(np.float64), ost,
                                 dl_dimage=dl.cpu().numpy().astype(np.float64))
        img = images.cpu().numpy().astype(np.float64)
        assert U.rel_err(img, op.fwd.image) <= 2e-4
        assert U.rel_err(grads.masks.cpu().numpy(), op.bwd.d_mask) <= 2e-3
        assert U.rel_err(grads.means.cpu().numpy(), op.grads.means) <= 2e-3
        del graph
    finally:
        rast.reserve(frame, 0)
        rast.release_frame(frame)
