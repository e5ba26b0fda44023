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


def test_captured_importance_forward_matches_eager(rast):
    """The importance forward inside a captured step: every replay (with eager
    work between) gives the eager images bit for bit, the eager maxima bit
    for bit and the eager sums up to the order of the FP64 atomics."""
    s = _multiview_scene()
    dev, params, cams, images, dl, grads = _setup(rast, s)
    n = params["means"].shape[0]
    isum, imax = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    frame = rast.acquire_frame()
    try:
        def step():
            rast.forward_importance(frame, params, dev["masks"], cams, images=images, imp_sum=isum, imp_max=imax)
            rast.backward(frame, params, dl, out=grads)

        step()
        rast.reserve(frame, 1.25)
        step()  # first call on the fixed workspace allocates the accumulator
        rast.check(frame)
        torch.cuda.synchronize()
        ref = (images.cpu().numpy().copy(), isum.cpu().numpy().copy(), imax.cpu().numpy().copy())
        assert np.count_nonzero(ref[1]) > 100
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for rep in range(3):
            isum.fill_(-1.0)
            imax.fill_(-1.0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            rast.check(frame)
            assert np.array_equal(images.cpu().numpy(), ref[0]), rep
            assert np.array_equal(imax.cpu().numpy(), ref[2]), rep
            assert U.rel_err(isum.cpu().numpy(), ref[1]) <= 1e-6, rep
            _ = (isum * 2.0).sum().item()
        del graph
    finally:
        rast.reserve(frame, 0)
        rast.release_frame(frame)


def test_captured_pruning_matches_eager():
    """Draws and compaction with a caller-provided scratch are capturable:
    replays reproduce the eager keep mask, kept count and compacted rows."""
    from paper_2412_20522_amd import maskgs as M
    ctx = M.mgs_create(0)
    n = 50_001
    rng = np.random.default_rng(21)
    scores = torch.from_numpy(scenegen.converged_mask_scores(n)).cuda()
    data = torch.from_numpy(rng.normal(size=(n, 7)).astype(np.float32)).cuda()
    keep = torch.empty(n, dtype=torch.int32, device="cuda")
    outs = [torch.empty_like(scores), torch.empty_like(data)]
    n_kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    scratch = torch.empty(int(M.lib().mgs_compact_scratch_bytes(n)), dtype=torch.uint8, device="cuda")

    def step():
        M.mgs_prune_sample(ctx, scores, 77, 500, 10, keep)
        M.mgs_compact_rows(ctx, keep, [scores, data], outs, n_kept=n_kept, scratch=scratch)

    step()
    torch.cuda.synchronize()
    k = int(n_kept.item())
    ref = [keep.cpu().numpy().copy(), outs[0][:k].cpu().numpy().copy(), outs[1][:k].cpu().numpy().copy()]
    assert np.array_equal(ref[0].astype(bool), oracle.prune_keep(scenegen.converged_mask_scores(n), 77, 500))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for o in outs:
            o.fill_(-3.0)
        n_kept.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(n_kept.item()) == k, rep
        assert np.array_equal(keep.cpu().numpy(), ref[0]), rep
        assert np.array_equal(outs[0][:k].cpu().numpy(), ref[1]), rep
        assert np.array_equal(outs[1][:k].cpu().numpy(), ref[2]), rep
    del graph
