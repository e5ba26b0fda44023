"""Pins of the oracle's mask-application variants (the ablations of Sec. 4.3):
mask x opacity (Table 7) and deterministic straight-through masks (Table 6).

Mask x opacity is pinned by central finite differences of its own forward,
by its reduction to masked rasterization where the two coincide (no alpha
filter, no clamp: alpha = M o G either way), and by the mechanism the paper
names for it: with the alpha filter on, an unsampled Gaussian is filtered out
and receives no gradient at all, where masked rasterization still gives it
dL/dM (Eq. 6).  The threshold masks are pinned by the closed form of the
inverse sigmoid and by finite differences of the soft value.
"""
import math

import numpy as np
import pytest

import scenegen

KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _scene(n, w, h, seed, deg=2, ls=-1.7, opacity_mean=-1.0):
    return scenegen.small_scene(n, w, h, seed=seed, sh_degree=deg, log_scale_mean=ls, depth=3.5,
                                opacity_mean=opacity_mean, n_views=1)


def _loss(orc, sc, cams, mask, st, w, mode):
    out = orc.run_pipeline(sc, cams, mask, st, backward=False, mask_mode=mode)
    return float(np.dot(out.fwd.image, w))


def test_opacity_mode_finite_differences(orc):
    sc = _scene(6, 20, 16, seed=31)
    st = orc.RasterSettings(sh_degree=2, bg=(0.4, 0.3, 0.8), exact_mode=True)
    cams = [sc["cameras"][0], scenegen.orbit_camera(3.2, 25.0, 10.0, 18, 14)]
    rng = np.random.default_rng(8)
    mask = rng.uniform(0.2, 1.0, 6)
    w = rng.normal(size=3 * (20 * 16 + 18 * 14))
    base = {k: np.asarray(sc[k], np.float64).copy() for k in KEYS}
    out = orc.run_pipeline(base, cams, mask, st, dl_dimage=w, mask_mode="opacity")
    h = 1e-6
    for key in ("opacity_logits", "means"):
        flat = base[key].reshape(-1)
        fd = np.zeros(flat.size)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp = _loss(orc, base, cams, mask, st, w, "opacity")
            flat[j] = old - h
            lm = _loss(orc, base, cams, mask, st, w, "opacity")
            flat[j] = old
            fd[j] = (lp - lm) / (2 * h)
        g = getattr(out.grads, key).reshape(-1)
        assert np.abs(fd - g).max() <= 2e-6 * max(np.abs(fd).max(), 1e-3), key
    fdm = np.zeros(6)
    for j in range(6):
        mp, mm = mask.copy(), mask.copy()
        mp[j] += h
        mm[j] -= h
        fdm[j] = (_loss(orc, base, cams, mp, st, w, "opacity") - _loss(orc, base, cams, mm, st, w, "opacity")) / (2 * h)
    assert np.abs(fdm).max() > 1e-3
    np.testing.assert_allclose(out.bwd.d_mask, fdm, rtol=1e-6, atol=1e-8)


def test_opacity_mode_reduces_to_masked_rasterization_without_filters(orc):
    """No alpha filter and no clamped alpha: both modes compute alpha = M o G,
    so images and every gradient agree, fractional masks included."""
    sc = _scene(40, 32, 24, seed=32)
    st = orc.RasterSettings(sh_degree=2, bg=(0.1, 0.5, 0.3), exact_mode=True)
    cam = sc["cameras"][0]
    rng = np.random.default_rng(9)
    mask = rng.uniform(0.0, 1.0, 40)
    w = rng.normal(size=3 * 32 * 24)
    a = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w, mask_mode="raster")
    b = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w, mask_mode="opacity")
    assert np.all(a.proj[0].opacity < 0.99)
    np.testing.assert_allclose(b.fwd.image, a.fwd.image, rtol=0, atol=1e-13)
    np.testing.assert_allclose(b.bwd.d_mask, a.bwd.d_mask, rtol=1e-9, atol=1e-13)
    for key in KEYS:
        ga, gb = getattr(a.grads, key), getattr(b.grads, key)
        np.testing.assert_allclose(gb, ga, rtol=1e-9, atol=1e-12 * max(np.abs(ga).max(), 1.0), err_msg=key)


def test_opacity_mode_starves_unsampled_gaussians(orc):
    """With the alpha filter on and binary masks the two modes render the same
    image, and sampled Gaussians get the same gradients; an unsampled one gets
    dL/dM = 0 under mask x opacity, but not under masked rasterization."""
    sc = _scene(60, 40, 32, seed=33)
    st = orc.RasterSettings(sh_degree=2, bg=(0.3, 0.3, 0.6))
    cam = sc["cameras"][0]
    rng = np.random.default_rng(10)
    mask = (rng.uniform(size=60) < 0.6).astype(np.float64)
    w = rng.normal(size=3 * 40 * 32)
    a = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w, mask_mode="raster")
    b = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w, mask_mode="opacity")
    assert np.all(a.proj[0].opacity < 0.99)
    np.testing.assert_allclose(b.fwd.image, a.fwd.image, rtol=0, atol=1e-15)
    off, on = mask == 0.0, mask == 1.0
    assert np.all(b.bwd.d_mask[off] == 0.0)
    assert np.count_nonzero(a.bwd.d_mask[off]) >= 0.5 * off.sum()
    np.testing.assert_allclose(b.bwd.d_mask[on], a.bwd.d_mask[on], rtol=1e-10, atol=1e-14)
    for key in KEYS:
        ga, gb = getattr(a.grads, key), getattr(b.grads, key)
        assert np.all(gb[off] == 0.0) and np.all(ga[off] == 0.0), key
        np.testing.assert_allclose(gb, ga, rtol=1e-10, atol=1e-13 * max(np.abs(ga).max(), 1.0), err_msg=key)


@pytest.mark.parametrize("thr", [0.01, 0.5, 0.9])
def test_threshold_masks_closed_form(orc, thr):
    """M = 1 exactly when s0 - s1 exceeds logit(threshold); y(s, s) = 1/2."""
    rng = np.random.default_rng(11)
    s = rng.normal(size=(5000, 2)) * 3.0
    gap = s[:, 0] - s[:, 1]
    cut = math.log(thr / (1.0 - thr))
    s = s[np.abs(gap - cut) > 1e-9]
    m, y = orc.threshold_masks(s, thr)
    assert np.array_equal(m, (s[:, 0] - s[:, 1] > cut).astype(np.float64))
    assert np.all((y > 0.0) & (y < 1.0))
    m2, y2 = orc.threshold_masks(np.array([[0.3, 0.3], [-2.0, -2.0]]), thr)
    assert np.all(y2 == 0.5) and np.all(m2 == float(0.5 > thr))


def test_threshold_masks_straight_through_gradient(orc):
    """mask_grad at tau = 1 on the threshold masks' soft value: dL/ds0 is
    dL/dM times dy/ds0 (by central differences), dL/ds1 its negative."""
    rng = np.random.default_rng(12)
    s = rng.normal(size=(64, 2)) * 2.0
    m, y = orc.threshold_masks(s, 0.01)
    d = rng.normal(size=64)
    g, _ = orc.mask_grad(d, m, y, 1.0, 0.0)
    h = 1e-6
    sp, sm = s.copy(), s.copy()
    sp[:, 0] += h
    sm[:, 0] -= h
    dy = (orc.threshold_masks(sp, 0.01)[1] - orc.threshold_masks(sm, 0.01)[1]) / (2 * h)
    np.testing.assert_allclose(g[:, 0], d * dy, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(g[:, 1], -g[:, 0], rtol=0, atol=0)
