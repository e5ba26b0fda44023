"""Stage-wise parity of the HIP path with the FP64 oracle.

Each stage runs on the GPU through its C-ABI entry point; the oracle stage
runs on the GPU's own upstream outputs widened exactly to FP64.  Integer
stages (tile counts, scan, keys, sort order, ranges, last blended entry,
entries examined) must match bit for bit; compositing within 1e-5 of the
image scale; gradients within 2e-3 relative.  Pixels whose discrete
decisions the oracle flags as within a relative margin of a threshold are
left out of element-wise checks (and the Gaussians they touch out of the
element-wise gradient checks); norm-wise checks include everything.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    M = U.M()
    c = M.mgs_create(0)
    yield c
    M.mgs_destroy(c)


def _scene(kind):
    if kind == "tiny":
        return scenegen.tiny_scene()
    if kind == "ragged_sh3":
        return scenegen.small_scene(3000, 150, 90, seed=101, sh_degree=3, log_scale_mean=-2.6)
    if kind == "ragged_sh1":
        return scenegen.small_scene(2500, 97, 61, seed=102, sh_degree=1, log_scale_mean=-2.4)
    if kind == "multiview":
        s = scenegen.small_scene(2000, 80, 60, seed=103, sh_degree=2, log_scale_mean=-2.5, n_views=3)
        s["cameras"][1] = scenegen.orbit_camera(4.0, 35.0, 8.0, 50, 72)
        s["cameras"][2] = scenegen.orbit_camera(3.5, -60.0, -12.0, 33, 29)
        return s
    if kind == "many":
        # 100,011 records: more than one group of 1024 waves in the list
        # offsets, and a ragged last workgroup of positions
        s = scenegen.small_scene(33_337, 160, 120, seed=104, sh_degree=1, log_scale_mean=-3.0, n_views=3)
        s["cameras"][1] = scenegen.orbit_camera(4.5, 25.0, 10.0, 144, 96)
        s["cameras"][2] = scenegen.orbit_camera(3.8, -40.0, -8.0, 101, 77)
        return s
    raise KeyError(kind)


def _run_stages(ctx, scene, cams, bg=(0.0, 0.0, 0.0), **kw):
    deg = scene["sh_degree"]
    ost, gst = U.settings_pair(sh_degree=deg, bg=bg, **kw)
    dev = U.to_device(scene)
    n = scene["means"].shape[0]
    rec, depth, radius, tiles = U.gpu_project(ctx, dev, cams, gst)
    offsets, K, keys, vals, ranges = U.gpu_lists(ctx, rec, depth, radius, tiles, n, cams, gst)
    oi = U.oracle_inputs_from_rec(rec)
    widths = [c["width"] for c in cams]
    heights = [c["height"] for c in cams]
    valid = (radius.cpu().numpy() > 0).astype(np.uint8)
    olists = oracle.build_lists(widths, heights, n, oi["mean2d"], radius.cpu().numpy().astype(np.float64),
                                U.u32(depth), valid, ost)
    return dict(ost=ost, gst=gst, dev=dev, n=n, rec=rec, depth=depth, radius=radius, tiles=tiles, offsets=offsets,
                K=K, keys=keys, vals=vals, ranges=ranges, oi=oi, olists=olists, widths=widths, heights=heights,
                masks=scene["masks"].astype(np.float64))


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["tiny", "ragged_sh3", "multiview"])
def test_project_matches_oracle(ctx, kind):
    s = _scene(kind)
    cams = s["cameras"]
    ost, gst = U.settings_pair(sh_degree=s["sh_degree"])
    dev = U.to_device(s)
    rec, depth, radius, tiles = U.gpu_project(ctx, dev, cams, gst)
    n = s["means"].shape[0]
    rec = rec.cpu().numpy().astype(np.float64)
    for v, cam in enumerate(cams):
        pr = oracle.project(s, cam, ost)
        sl = slice(v * n, (v + 1) * n)
        gvalid = radius.cpu().numpy()[sl] > 0
        assert np.array_equal(gvalid, pr.valid.astype(bool))
        # depth keys agree bit for bit end to end
        assert np.array_equal(U.u32(depth)[sl][gvalid], pr.depth_bits[gvalid])
        r = rec[sl][gvalid]
        np.testing.assert_allclose(r[:, 0:2], pr.mean2d[gvalid], rtol=0, atol=2e-4 * max(cam["width"], 1) / 100)
        scale = np.abs(pr.conic[gvalid]).max(axis=1, keepdims=True)
        np.testing.assert_allclose(U.conic_from_rec(r) / scale, pr.conic[gvalid] / scale, rtol=0, atol=5e-5)
        np.testing.assert_allclose(r[:, 5], pr.opacity[gvalid], rtol=2e-6)
        np.testing.assert_allclose(r[:, 8:11], pr.color[gvalid], rtol=0, atol=5e-6)
        np.testing.assert_array_equal(r[:, 6], s["masks"][gvalid])
        # radii (ceil of a double-precision expression, stored in FP32) agree exactly
        mism = np.count_nonzero(radius.cpu().numpy()[sl][gvalid] != pr.radius[gvalid].astype(np.float32))
        assert mism == 0, mism


def _rect_mismatches(s, ctx):
    """Projected records of the GPU (FP32 storage of a double-precision
    chain) against the oracle's FP64 projection: validity, radius and tile
    rectangle of every record, the rectangle taken in double from the FP32
    centre and radius on both sides (the GPU's storage precision)."""
    cams = s["cameras"]
    ost, gst = U.settings_pair(sh_degree=s["sh_degree"])
    dev = U.to_device(s, np.ones(s["means"].shape[0], np.float32))
    rec, depth, radius, tiles = U.gpu_project(ctx, dev, cams, gst)
    n = s["means"].shape[0]
    rec = rec.cpu().numpy()
    rad = radius.cpu().numpy()
    out = {"records": 0, "valid": 0, "radius": 0, "rect": 0, "tiles": 0}
    for v, cam in enumerate(cams):
        pr = oracle.project(s, cam, ost)
        sl = slice(v * n, (v + 1) * n)
        gvalid = rad[sl] > 0
        ovalid = pr.valid.astype(bool)
        out["records"] += n
        out["valid"] += int(np.count_nonzero(gvalid != ovalid))
        both = gvalid & ovalid
        gr = rad[sl][both].astype(np.float64)
        orr = pr.radius[both].astype(np.float32).astype(np.float64)
        out["radius"] += int(np.count_nonzero(gr != orr))
        gw, gh = (cam["width"] + 15) // 16, (cam["height"] + 15) // 16
        a = tile_rects(rec[sl][both, 0].astype(np.float64), rec[sl][both, 1].astype(np.float64), gr, gw, gh, 16, 16)
        b = tile_rects(pr.mean2d[both, 0].astype(np.float32).astype(np.float64),
                       pr.mean2d[both, 1].astype(np.float32).astype(np.float64), orr, gw, gh, 16, 16)
        out["rect"] += int(np.count_nonzero(np.any(np.stack(a) != np.stack(b), axis=0)))
        ot = np.zeros(n, np.int64)
        ot_both = np.maximum(b[2] - b[0] + 1, 0) * np.maximum(b[3] - b[1] + 1, 0)
        ot[both] = ot_both.astype(np.int64)
        out["tiles"] += int(np.count_nonzero(U.u32(tiles)[sl].astype(np.int64) != ot))
    return out


@pytest.mark.parametrize("kind", ["tiny", "object", "unbounded"])
def test_projection_mismatches_counted_at_full_size(ctx, kind):
    """Radius and rectangle mismatches between the GPU projection and the
    oracle's, counted over every record of the tiny (4096), object (200k)
    and unbounded (1.5M, heavy-tailed scales including splats wider than
    FP32 holds) workloads: none."""
    s = {"tiny": scenegen.tiny_scene, "object": scenegen.object_scene, "unbounded": scenegen.unbounded_scene}[kind]()
    out = _rect_mismatches(s, ctx)
    print(kind, out)
    assert out["valid"] == 0 and out["radius"] == 0 and out["rect"] == 0 and out["tiles"] == 0, out


def test_tiles_and_lists_match_oracle_bitwise(ctx):
    for kind in ["tiny", "ragged_sh3", "multiview"]:
        s = _scene(kind)
        for tw, th in [(16, 16), (8, 8), (32, 8)]:
            r = _run_stages(ctx, s, s["cameras"], tile_w=tw, tile_h=th, fwd_ppt=1, bwd_ppt=1)
            ol = r["olists"]
            assert np.array_equal(U.u32(r["tiles"]).astype(np.int64), ol.tiles_touched)
            assert r["K"] == ol.keys.size
            assert np.array_equal(U.u64(r["keys"]), ol.keys)
            assert np.array_equal(U.u32(r["vals"]), ol.vals)
            # non-empty ranges are unique; an empty tile may be any [x, x)
            gr = U.u32(r["ranges"]).reshape(-1, 2)
            nonempty = ol.ranges[:, 1] > ol.ranges[:, 0]
            assert np.array_equal(gr[nonempty], ol.ranges[nonempty])
            assert np.all(gr[~nonempty, 0] == gr[~nonempty, 1])


def tile_rects(u, v, r, gw, gh, tw, th):
    """Inclusive tile rectangle of each record's square footprint
    [u - r, u + r] x [v - r, v + r], clamped to the grid (empty when
    x0 > x1 or y0 > y1), in FP64 like the tile assignment of Sec. 3.1."""
    x0 = np.maximum(np.floor((u - r) / tw), 0)
    x1 = np.minimum(np.floor((u + r) / tw), gw - 1)
    y0 = np.maximum(np.floor((v - r) / th), 0)
    y1 = np.minimum(np.floor((v + r) / th), gh - 1)
    return x0, y0, x1, y1


def merged_tile_lists(cams, tw, th, vals, ranges, order, depth_bits, mean2d, radius, wide_mask):
    """Per-tile lists of the hybrid binning as record ids: the tile's own
    entries (positions into `order`) merged with the entries of its region
    (MGS_REGION_TILES^2 tiles) whose tile rectangle contains the tile, in
    (depth bits, record) order.  Also returns the records listed per region."""
    RG = U.M().REGION_TILES
    T = sum(((c["width"] + tw - 1) // tw) * ((c["height"] + th - 1) // th) for c in cams)
    out, region_recs = [], []
    roff = 0
    n = wide_mask.size // len(cams)
    for v, c in enumerate(cams):
        gw, gh = (c["width"] + tw - 1) // tw, (c["height"] + th - 1) // th
        rw, rh = (gw + RG - 1) // RG, (gh + RG - 1) // RG
        # every wide record of the view once in each region its rectangle overlaps
        wr = v * n + np.nonzero(wide_mask[v * n:(v + 1) * n])[0]
        x0, y0, x1, y1 = tile_rects(mean2d[wr, 0], mean2d[wr, 1], radius[wr], gw, gh, tw, th)
        want = int(((x1 // RG - x0 // RG + 1) * (y1 // RG - y0 // RG + 1)).sum())
        got = int(sum(ranges[T + roff + k, 1] - ranges[T + roff + k, 0] for k in range(rw * rh)))
        assert got == want, (v, got, want)
        for ry in range(rh):
            for rx in range(rw):
                rg = T + roff + ry * rw + rx
                recs = order[vals[ranges[rg, 0]:ranges[rg, 1]]].astype(np.int64)
                x0, y0, x1, y1 = tile_rects(mean2d[recs, 0], mean2d[recs, 1], radius[recs], gw, gh, tw, th)
                # a region lists wide records whose rectangle overlaps it, each once
                assert np.all((x0 // RG <= rx) & (rx <= x1 // RG) & (y0 // RG <= ry) & (ry <= y1 // RG))
                assert np.all(wide_mask[recs]) and np.unique(recs).size == recs.size
                region_recs.append(recs)
        for ty in range(gh):
            for tx in range(gw):
                t = len(out)
                narrow = order[vals[ranges[t, 0]:ranges[t, 1]]].astype(np.int64)
                rg = T + roff + (ty // RG) * rw + tx // RG
                cand = order[vals[ranges[rg, 0]:ranges[rg, 1]]].astype(np.int64)
                x0, y0, x1, y1 = tile_rects(mean2d[cand, 0], mean2d[cand, 1], radius[cand], gw, gh, tw, th)
                cover = (x0 <= tx) & (tx <= x1) & (y0 <= ty) & (ty <= y1)
                recs = np.concatenate([narrow, cand[cover]])
                perm = np.lexsort((recs, depth_bits[recs].astype(np.int64)))
                out.append(recs[perm])
        roff += rw * rh
    return out, region_recs


@pytest.mark.parametrize("kind", ["tiny", "ragged_sh3", "multiview", "many"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
@pytest.mark.parametrize("wide_tiles", [-1, 0, 1])
def test_whole_path_lists_match_oracle_bitwise(ctx, kind, tile, wide_tiles):
    """mgs_forward bins in depth order, duplicates only records with few
    tiles and keeps the others once per view in a wide list; the per-tile
    merge of the two must equal the oracle's (tile, depth, record) lists
    exactly, and the last blended entry and entries examined per pixel (as
    indices into the merged list) must equal the oracle's."""
    M = U.M()
    s = _scene(kind)
    cams = s["cameras"]
    tw, th = tile
    bg = (0.3, 0.5, 0.7)
    ost, gst = U.settings_pair(sh_degree=s["sh_degree"], tile_w=tw, tile_h=th, fwd_ppt=1, bwd_ppt=1,
                               wide_tiles=wide_tiles, batch_depth=64, bg=bg, tile_cull=0)
    dev = U.to_device(s)
    frame = M.mgs_frame_create(ctx)
    try:
        P = sum(c["width"] * c["height"] for c in cams)
        img = torch.empty(3 * P, device="cuda")
        M.mgs_forward(ctx, frame, U.gstruct(dev), cams, gst, img)
        ex = {k: M.mgs_frame_export(ctx, frame, k) for k in
              ("records", "radius", "depth", "tiles", "values", "ranges", "order", "last", "stats", "t_final")}
        st = M.mgs_frame_get_stats(frame)
        torch.cuda.synchronize()
    finally:
        M.mgs_frame_destroy(frame)
    n = s["means"].shape[0]
    rec = ex["records"].view(-1, 12)
    oi = U.oracle_inputs_from_rec(rec)
    rad = ex["radius"].cpu().numpy().astype(np.float64)
    dbits = U.u32(ex["depth"])
    ol = oracle.build_lists([c["width"] for c in cams], [c["height"] for c in cams], n, oi["mean2d"], rad, dbits,
                            (rad > 0).astype(np.uint8), ost)
    # records covering more tiles than the threshold are listed per region
    thr = {-1: None, 0: 64, 1: 1}[wide_tiles]
    ntiles = U.u32(ex["tiles"]).astype(np.int64)
    want_wide = np.zeros(ntiles.size, bool) if thr is None else ntiles > thr
    assert st["n_wide"] == int(want_wide.sum())
    if wide_tiles < 0:
        assert st["n_wide"] == 0
    if wide_tiles == 1:
        assert st["n_wide"] > 0
    lists, region_recs = merged_tile_lists(cams, tw, th, U.u32(ex["values"]), U.u32(ex["ranges"]).reshape(-1, 2),
                                           U.u32(ex["order"]), dbits, oi["mean2d"], rad, want_wide)
    listed = np.unique(np.concatenate(region_recs)) if region_recs else np.zeros(0, np.int64)
    assert np.array_equal(listed, np.nonzero(want_wide)[0])
    assert len(lists) == ol.ranges.shape[0]
    assert st["n_instances"] == U.u32(ex["values"]).size
    rg = U.u32(ex["ranges"]).reshape(-1, 2).astype(np.int64)
    assert int((rg[:, 1] - rg[:, 0]).sum()) == st["n_instances"]  # every entry in exactly one cell
    for t, lst in enumerate(lists):
        a, b = ol.ranges[t]
        assert np.array_equal(lst, ol.vals[a:b].astype(np.int64)), t
    # per pixel: last blended entry and entries examined, local to the tile list
    of = oracle.render_fwd([c["width"] for c in cams], [c["height"] for c in cams], n, oi["mean2d"], oi["conic"],
                           oi["opacity"], oi["color"], s["masks"].astype(np.float64), ol, ost)
    ok = of.flags == 0
    assert ok.mean() > 0.99
    start = np.empty(P, np.int64)
    off = 0
    toff = 0
    for c in cams:
        w, h = c["width"], c["height"]
        gw = (w + tw - 1) // tw
        yy, xx = np.divmod(np.arange(w * h), w)
        start[off:off + w * h] = ol.ranges[toff + (yy // th) * gw + xx // tw, 0]
        off += w * h
        toff += gw * ((h + th - 1) // th)
    o_last = np.where(of.last >= 0, of.last - start, -1)
    assert np.array_equal(ex["last"].cpu().numpy()[ok], o_last[ok])
    stats = ex["stats"].cpu().numpy().reshape(-1, 4)
    assert np.array_equal(stats[ok, 0], of.examined[ok])
    assert np.abs(ex["t_final"].cpu().numpy() - of.t_final)[ok].max() <= 1e-5
    gi = img.cpu().numpy().astype(np.float64)
    assert U.rel_err(gi, of.image) <= 1e-4


# ---------------------------------------------------------------------------
# scan and sort on synthetic inputs (bit-exact against the definitions)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 7, 4095, 4096, 4097, 123457])
def test_scan_matches_cumsum(ctx, n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 300, n).astype(np.uint32)
    inp = torch.from_numpy(a.view(np.int32)).cuda()
    out = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    U.M().mgs_scan(ctx, inp, out[:n], total)
    torch.cuda.synchronize()
    want = np.concatenate([[0], np.cumsum(a.astype(np.uint64))[:-1]]) if n else np.zeros(0)
    assert np.array_equal(U.u32(out[:n]).astype(np.uint64), want.astype(np.uint64))
    assert int(total.item()) == int(a.astype(np.uint64).sum())


@pytest.mark.parametrize("K,bits", [(2, 40), (4096, 38), (4097, 46), (100_001, 47), (300_000, 64),
                                    (9_000_003, 48)])
def test_sort_is_stable_and_matches_lexsort(ctx, K, bits):
    rng = np.random.default_rng(K)
    tiles = rng.integers(0, 1 << max(bits - 32, 0), K, dtype=np.uint64) if bits > 32 else np.zeros(K, np.uint64)
    depth = rng.integers(0, 1 << 31, K, dtype=np.uint64)
    depth[::7] = depth[0]  # many equal keys: order must follow the input
    keys = (tiles << np.uint64(32)) | depth
    if bits == 64:
        keys = rng.integers(0, 2 ** 63, K, dtype=np.uint64) * np.uint64(2) + (keys & np.uint64(1))
        keys[::5] = keys[1]
    vals = np.arange(K, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    U.M().mgs_sort(ctx, kt, vt, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(U.u64(kt), keys[order])
    assert np.array_equal(U.u32(vt), vals[order])


# ---------------------------------------------------------------------------
# compositing, stage-wise
# ---------------------------------------------------------------------------

SHAPES = [(16, 16, 1, 1, 256), (16, 16, 2, 4, 128), (16, 16, 4, 4, 64), (8, 8, 1, 1, 32), (16, 8, 2, 1, 256),
          (32, 8, 4, 2, 128)]


def _product_run(ctx, s, shape, cull, wide, persistent, bg, dl_seed=7):
    """The whole path (mgs_forward / mgs_backward, the product kernels) in a
    given compositing configuration; exports of the frame, the image, the
    per-record 2D gradients and the mask gradients."""
    M = U.M()
    tw, th, fppt, bppt, batch = shape
    cams = s["cameras"]
    ost, gst = U.settings_pair(sh_degree=s["sh_degree"], tile_w=tw, tile_h=th, fwd_ppt=fppt, bwd_ppt=bppt,
                               batch_depth=batch, bg=bg, tile_cull=cull, wide_tiles=wide, persistent=persistent,
                               stats=1)
    dev = U.to_device(s)
    n = s["means"].shape[0]
    P = sum(c["width"] * c["height"] for c in cams)
    R = n * len(cams)
    frame = M.mgs_frame_create(ctx)
    try:
        img = torch.full((3 * P,), -7.0, device="cuda")
        tfin = torch.full((P,), -7.0, device="cuda")
        M.mgs_forward(ctx, frame, U.gstruct(dev), cams, gst, img, tfin)
        ex = {k: M.mgs_frame_export(ctx, frame, k) for k in ("records", "radius", "depth", "last", "stats")}
        dl = np.random.default_rng(dl_seed).normal(size=3 * P).astype(np.float32)
        d_rec = torch.full((max(R, 1), 9), 5.0, device="cuda")
        d_masks = torch.full((max(n, 1),), 5.0, device="cuda")
        gr = M.gradients_struct(d_masks=d_masks, d_records=d_rec)
        M.mgs_backward(ctx, frame, torch.from_numpy(dl).cuda(), gr)
        torch.cuda.synchronize()
    finally:
        M.mgs_frame_destroy(frame)
    oi = U.oracle_inputs_from_rec(ex["records"].view(-1, 12))
    rad = ex["radius"].cpu().numpy().astype(np.float64)
    ws, hs = [c["width"] for c in cams], [c["height"] for c in cams]
    ol = oracle.build_lists(ws, hs, n, oi["mean2d"], rad, U.u32(ex["depth"]), (rad > 0).astype(np.uint8), ost)
    return dict(img=img.cpu().numpy().astype(np.float64), tfin=tfin.cpu().numpy(), ex=ex, dl=dl, ost=ost, oi=oi,
                ol=ol, n=n, P=P, ws=ws, hs=hs, d_rec=d_rec[:R].cpu().numpy().astype(np.float64),
                d_masks=d_masks[:n].cpu().numpy().astype(np.float64), masks=s["masks"].astype(np.float64))


def _pixel_channels(ok, ws, hs):
    out, off = [], 0
    for w, h in zip(ws, hs):
        out.append(np.tile(ok[off:off + w * h], 3))
        off += w * h
    return np.concatenate(out)


@pytest.mark.parametrize("kind", ["tiny", "ragged_sh3", "multiview"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("cull", [0, 1])
def test_product_compositing_matches_oracle(ctx, kind, shape, cull):
    """Forward and backward compositing of the whole path (the kernels the
    product runs) against the oracle's compositing on the GPU's own records
    and the lists of Sec. 3.1, element-wise: images and final transmittance
    on unflagged pixels; per pixel the last blended entry (lists without
    culling); per-record dL/d(u, v), conic (stored basis), opacity, colour
    and per-Gaussian dL/dM on Gaussians that touch no flagged pixel."""
    s = _scene(kind)
    bg = (0.0, 0.0, 0.0) if kind == "tiny" else (0.3, 0.5, 0.7)
    wide = {0: -1, 1: 0}[SHAPES.index(shape) % 2] if kind != "multiview" else 1
    r = _product_run(ctx, s, shape, cull, wide, persistent=SHAPES.index(shape) % 2, bg=bg)
    oi, ol, ost = r["oi"], r["ol"], r["ost"]
    of = oracle.render_fwd(r["ws"], r["hs"], r["n"], oi["mean2d"], oi["conic"], oi["opacity"], oi["color"],
                           r["masks"], ol, ost)
    ok = of.flags == 0
    assert ok.mean() > 0.99
    scale = max(np.abs(of.image).max(), 1.0)
    err = np.abs(r["img"] - of.image)[_pixel_channels(ok, r["ws"], r["hs"])].max()
    assert err <= 1e-5 * scale, err
    assert np.abs(r["tfin"] - of.t_final)[ok].max() <= 1e-5
    assert U.rel_err(r["img"], of.image) <= 1e-4
    if not cull:
        tw, th = shape[0], shape[1]
        start = np.empty(r["P"], np.int64)
        off = toff = 0
        for w, h in zip(r["ws"], r["hs"]):
            gw = (w + tw - 1) // tw
            yy, xx = np.divmod(np.arange(w * h), w)
            start[off:off + w * h] = ol.ranges[toff + (yy // th) * gw + xx // tw, 0]
            off += w * h
            toff += gw * ((h + th - 1) // th)
        o_last = np.where(of.last >= 0, of.last - start, -1)
        assert np.array_equal(r["ex"]["last"].cpu().numpy()[ok], o_last[ok])
        stats = r["ex"]["stats"].cpu().numpy().reshape(-1, 4)
        assert np.array_equal(stats[ok, 0], of.examined[ok])
    ob = oracle.render_bwd(r["ws"], r["hs"], r["n"], oi["mean2d"], oi["conic"], oi["opacity"], oi["color"],
                           r["masks"], ol, r["dl"].astype(np.float64), ost)
    g = r["d_rec"]
    exr = ob.touched_flagged.astype(bool)
    rec64 = r["ex"]["records"].view(-1, 12).cpu().numpy().astype(np.float64)
    U.assert_grad_close(g[:, 0:2], ob.d_mean2d, exr, name="mean2d")
    U.assert_grad_close(g[:, 2:5], U.dstable_from_dabc(rec64[:, 2], rec64[:, 3], ob.d_conic), exr, name="conic")
    U.assert_grad_close(g[:, 5], ob.d_opacity, exr, name="opacity")
    U.assert_grad_close(g[:, 6:9], ob.d_color, exr, name="color")
    n = r["n"]
    U.assert_grad_close(r["d_masks"], ob.d_mask, exr.reshape(-1, n).any(axis=0), name="mask")
    # masked Gaussians receive a mask gradient and nothing else
    masked = r["masks"] == 0
    assert np.all(g.reshape(-1, n, 9)[:, masked, :] == 0.0)
    assert np.count_nonzero(r["d_masks"][masked]) > 0


@pytest.mark.parametrize("kind", ["tiny", "ragged_sh3", "multiview", "many"])
def test_culled_lists_keep_every_entry_that_can_blend(ctx, kind):
    """With tile culling the whole path lists a record in a tile (or its
    region) only where it can pass the per-pixel filters.  Checked on the
    exported lists against the oracle's lists of Sec. 3.1: every entry kept
    for a tile is in the oracle's list of that tile, and every oracle entry
    left out fails Q <= 9 or alpha >= 1/255 at every pixel centre of the
    tile (FP64, the GPU's own records)."""
    M = U.M()
    s = _scene(kind)
    cams = s["cameras"]
    RG = M.REGION_TILES
    for tw, th in [(16, 16), (8, 8)]:
        ost, gst = U.settings_pair(sh_degree=s["sh_degree"], tile_w=tw, tile_h=th, fwd_ppt=1, bwd_ppt=1,
                                   wide_tiles=4, batch_depth=64, tile_cull=1)
        dev = U.to_device(s)
        frame = M.mgs_frame_create(ctx)
        try:
            P = sum(c["width"] * c["height"] for c in cams)
            img = torch.empty(3 * P, device="cuda")
            M.mgs_forward(ctx, frame, U.gstruct(dev), cams, gst, img)
            ex = {k: M.mgs_frame_export(ctx, frame, k) for k in ("records", "radius", "depth", "values", "ranges",
                                                                   "order")}
            torch.cuda.synchronize()
        finally:
            M.mgs_frame_destroy(frame)
        n = s["means"].shape[0]
        rec = ex["records"].view(-1, 12).cpu().numpy().astype(np.float64)
        oi = U.oracle_inputs_from_rec(ex["records"].view(-1, 12))
        rad = ex["radius"].cpu().numpy().astype(np.float64)
        ol = oracle.build_lists([c["width"] for c in cams], [c["height"] for c in cams], n, oi["mean2d"], rad,
                                U.u32(ex["depth"]), (rad > 0).astype(np.uint8), ost)
        vals, order = U.u32(ex["values"]), U.u32(ex["order"])
        ranges = U.u32(ex["ranges"]).reshape(-1, 2).astype(np.int64)
        T = ol.ranges.shape[0]
        t = roff = 0
        dropped_total = kept_total = 0
        for c in cams:
            gw, gh = (c["width"] + tw - 1) // tw, (c["height"] + th - 1) // th
            rw = (gw + RG - 1) // RG
            for ty in range(gh):
                for tx in range(gw):
                    own = order[vals[ranges[t, 0]:ranges[t, 1]]].astype(np.int64)
                    rg = T + roff + (ty // RG) * rw + tx // RG
                    reg = order[vals[ranges[rg, 0]:ranges[rg, 1]]].astype(np.int64)
                    a, b = ol.ranges[t]
                    full = ol.vals[a:b].astype(np.int64)
                    assert np.all(np.isin(own, full)), (tw, t)
                    kept = np.union1d(own, reg)
                    drop = np.setdiff1d(full, kept)
                    kept_total += np.intersect1d(full, kept).size
                    dropped_total += drop.size
                    if drop.size:
                        x0, y0 = tx * tw, ty * th
                        xs = np.arange(x0, min(x0 + tw, c["width"])) + 0.5
                        ys = np.arange(y0, min(y0 + th, c["height"])) + 0.5
                        px, py = np.meshgrid(xs, ys)
                        dx = rec[drop, 0][:, None] - px.reshape(-1)[None, :]
                        dy = rec[drop, 1][:, None] - py.reshape(-1)[None, :]
                        A, B, C = (oi["conic"][drop, k][:, None] for k in range(3))
                        Q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
                        alpha = np.minimum(0.99, rec[drop, 5][:, None] * np.exp(-0.5 * Q))
                        can = (Q <= 9.0) & (alpha >= np.float32(1 / 255))
                        assert not can.any(), (tw, t, int(can.sum()))
                    t += 1
            roff += rw * ((gh + RG - 1) // RG)
        assert t == T
        # culling removes a real share of the entries, and keeps most
        assert dropped_total > 0 and kept_total > 0
        print(kind, (tw, th), "kept", kept_total, "dropped", dropped_total)


def test_project_backward_matches_oracle(ctx):
    for kind in ["tiny", "ragged_sh3", "multiview"]:
        s = _scene(kind)
        cams = s["cameras"]
        ost, gst = U.settings_pair(sh_degree=s["sh_degree"])
        dev = U.to_device(s)
        n = s["means"].shape[0]
        R = n * len(cams)
        rng = np.random.default_rng(11)
        d_rec = rng.normal(size=(R, 9)) * np.array([1.0, 1.0, 50.0, 50.0, 50.0, 0.5, 0.3, 0.3, 0.3])
        d_rec_t = torch.from_numpy(d_rec.astype(np.float32)).cuda()
        out = {k: torch.full_like(dev[k], 9.0) for k in U.PARAM_KEYS}
        gr = U.M().gradients_struct(out["means"], out["log_scales"], out["quats"], out["opacity_logits"], out["sh"])
        U.M().mgs_project_backward(ctx, U.gstruct(dev), cams, gst, d_rec_t, gr)
        torch.cuda.synchronize()
        dr = d_rec.astype(np.float32).astype(np.float64)
        # the kernel reads the conic gradient w.r.t. the stored (a, beta, gamma)
        prs = [oracle.project(s, c, ost) for c in cams]
        conic = np.concatenate([np.where(p.valid[:, None] > 0, p.conic, 1.0) for p in prs])
        dabc = U.dabc_from_dstable(conic, dr[:, 2:5])
        og = oracle.project_bwd(s, cams, ost, dr[:, 0:2], dabc, dr[:, 5], dr[:, 6:9])
        for k, o in [("means", og.means), ("log_scales", og.log_scales), ("quats", og.quats),
                     ("opacity_logits", og.opacity_logits), ("sh", og.sh)]:
            U.assert_grad_close(out[k].cpu().numpy().astype(np.float64), o, name=f"{kind}:{k}")


# ---------------------------------------------------------------------------
# masks, loss, optimiser
# ---------------------------------------------------------------------------

def test_sample_masks_match_oracle(ctx):
    rng = np.random.default_rng(3)
    n = 200_003
    scores = rng.normal(size=(n, 2)).astype(np.float32)
    st = torch.from_numpy(scores).cuda()
    m = torch.empty(n, device="cuda")
    y = torch.empty(n, device="cuda")
    for seed, step in [(0, 0), (2412, 17), (2 ** 40 + 5, 2 ** 33 + 1)]:
        U.M().mgs_sample_masks(ctx, st, 0.5, seed, step, m, y)
        torch.cuda.synchronize()
        om, oy = oracle.sample_masks(scores, 0.5, seed, step)
        assert np.array_equal(m.cpu().numpy().astype(np.float64), om)
        np.testing.assert_allclose(y.cpu().numpy(), oy, rtol=0, atol=1e-7)


def test_mask_grad_l1_and_adam_match_oracle(ctx):
    rng = np.random.default_rng(4)
    n = 50_001
    dM = rng.normal(size=n).astype(np.float32)
    mh = (rng.uniform(size=n) < 0.7).astype(np.float32)
    y = rng.uniform(0.01, 0.99, n).astype(np.float32)
    d = torch.empty(n, 2, device="cuda")
    lm = torch.zeros(1, device="cuda")
    U.M().mgs_mask_grad(ctx, torch.from_numpy(dM).cuda(), torch.from_numpy(mh).cuda(), torch.from_numpy(y).cuda(),
                        0.5, 0.1, d, lm)
    torch.cuda.synchronize()
    od, olm = oracle.mask_grad(dM, mh, y, 0.5, 0.1)
    np.testing.assert_allclose(d.cpu().numpy(), od, rtol=2e-6, atol=1e-9)
    assert abs(lm.item() - olm) <= 1e-6 * olm
    img = rng.uniform(size=30_000).astype(np.float32)
    tgt = rng.uniform(size=30_000).astype(np.float32)
    tgt[:10] = img[:10]
    di = torch.empty(30_000, device="cuda")
    loss = torch.zeros(1, device="cuda")
    U.M().mgs_l1_loss_grad(ctx, torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda(), di, loss)
    torch.cuda.synchronize()
    ol, od = oracle.l1_loss(img.astype(np.float64), tgt)
    assert np.array_equal(di.cpu().numpy().astype(np.float64), od.astype(np.float32).astype(np.float64))
    assert abs(loss.item() - ol) <= 1e-6 * ol
    p = rng.normal(size=1000).astype(np.float32)
    pt = torch.from_numpy(p.copy()).cuda()
    mt = torch.zeros(1000, device="cuda")
    vt = torch.zeros(1000, device="cuda")
    po = p.astype(np.float64)
    m1, m2 = np.zeros(1000), np.zeros(1000)
    for step in range(1, 4):
        g = rng.normal(size=1000).astype(np.float32)
        U.M().mgs_adam_step(ctx, pt, torch.from_numpy(g).cuda(), mt, vt, 1e-2, 0.9, 0.999, 1e-15, step)
        oracle.adam(po, g.astype(np.float64), m1, m2, 1e-2, 0.9, 0.999, 1e-15, step)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("m,offset", [(30_001, 0), (30_003, 0), (7, 0), (30_000, 1), (1, 0)])
def test_l1_loss_tails_and_misaligned_views(ctx, m, offset):
    """Lengths that leave a tail after the four-wide loop, and views one
    float off the 16-byte alignment (the scalar loop alone)."""
    rng = np.random.default_rng(m + offset)
    img = rng.uniform(size=m).astype(np.float32)
    tgt = rng.uniform(size=m).astype(np.float32)
    tgt[: min(3, m)] = img[: min(3, m)]
    bi = torch.zeros(m + offset, device="cuda")
    bt = torch.zeros(m + offset, device="cuda")
    bd = torch.full((m + offset,), 9.0, device="cuda")
    bi[offset:] = torch.from_numpy(img).cuda()
    bt[offset:] = torch.from_numpy(tgt).cuda()
    loss = torch.zeros(1, device="cuda")
    U.M().mgs_l1_loss_grad(ctx, bi[offset:], bt[offset:], bd[offset:], loss)
    torch.cuda.synchronize()
    ol, od = oracle.l1_loss(img.astype(np.float64), tgt)
    assert abs(float(loss.item()) - ol) <= 1e-6 * max(ol, 1e-30)
    assert np.array_equal(bd[offset:].cpu().numpy(), od.astype(np.float32))
