"""Pins of the oracle's importance by-products: per Gaussian, the sum and the
maximum over pixels of its blending weight M_i alpha_i T_i (the alpha T that
score-based pruning ranks by, Sec. 2; the factor Eq. 6 carries, Sec. 3.4).

Pinned by the telescoping identity of front-to-back compositing (per pixel
the weights and the final transmittance add up to 1, with the final
transmittance taken from the forward), by the five-splat one-pixel example
of Fig. 1 expanded by hand, and by a brute-force evaluation of a single
splat over the pixel grid in numpy.
"""
import math

import numpy as np

import scenegen


def test_weights_and_final_transmittance_add_up_to_one(orc):
    sc = scenegen.small_scene(400, 48, 40, seed=41, sh_degree=1, log_scale_mean=-2.0, n_views=2)
    cams = sc["cameras"]
    st = orc.RasterSettings(sh_degree=1, bg=(0.2, 0.3, 0.4))
    rng = np.random.default_rng(13)
    mask = rng.uniform(0.0, 1.0, 400)
    mask[::4] = 0.0
    out = orc.run_pipeline(sc, cams, mask, st, backward=False)
    s, m = orc.scene_importance(sc, cams, mask, st)
    P = out.fwd.t_final.size
    assert abs(s.sum() - (P - out.fwd.t_final.sum())) <= 1e-10 * P
    assert np.all(s[mask == 0.0] == 0.0) and np.all(m[mask == 0.0] == 0.0)
    assert np.all(m <= s + 1e-15) and np.all(m <= 0.99)
    assert np.count_nonzero(s) > 100


def test_fig1_five_splats_one_pixel(orc):
    """Five splats on the optical axis of a 1x1 image (G = 1 at the pixel
    centre, so alpha_i = o_i), the second and fifth masked:
    w_i = M_i o_i prod_{j < i} (1 - M_j o_j)."""
    cam = scenegen.camera_from_pose(np.eye(3), np.zeros(3), 1, 1)
    depths = [2.0, 3.0, 4.0, 5.0, 6.0]
    logits = np.array([0.2, -0.4, 0.9, -0.1, 0.5], np.float32)
    y00 = 0.5 / math.sqrt(math.pi)
    sc = dict(means=np.array([[0, 0, d] for d in depths], np.float32),
              log_scales=np.full((5, 3), math.log(0.01), np.float32),
              quats=np.tile(np.array([1, 0, 0, 0], np.float32), (5, 1)),
              opacity_logits=logits, sh=np.full((5, 1, 3), 0.1 / y00, np.float32))
    st = orc.RasterSettings(sh_degree=0)
    M = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    s, m = orc.scene_importance(sc, [cam], M, st)
    o = 1.0 / (1.0 + np.exp(-logits.astype(np.float64)))
    T, want = 1.0, np.zeros(5)
    for i in range(5):
        want[i] = M[i] * o[i] * T
        T *= 1.0 - M[i] * o[i]
    np.testing.assert_allclose(s, want, rtol=1e-13, atol=0)
    np.testing.assert_allclose(m, want, rtol=1e-13, atol=0)


def test_single_splat_brute_force(orc):
    """One splat alone (T = 1 everywhere): its weights are its alphas, so the
    sum and maximum are those of min(o exp(-Q/2), alpha_max) over the pixel
    centres that pass Q <= q_max and alpha >= alpha_min."""
    W, H = 64, 48
    cam = scenegen.camera_from_pose(np.eye(3), np.zeros(3), W, H)
    sc = dict(means=np.array([[0.13, -0.07, 3.0]], np.float32),
              log_scales=np.array([[math.log(0.25), math.log(0.1), math.log(0.15)]], np.float32),
              quats=np.array([[0.9, 0.2, -0.3, 0.1]], np.float32),
              opacity_logits=np.array([1.5], np.float32),
              sh=np.zeros((1, 1, 3), np.float32))
    st = orc.RasterSettings(sh_degree=0)
    proj = orc.project(sc, cam, st)
    u, v = proj.mean2d[0]
    a, b, c = proj.conic[0]
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dx, dy = u - X, v - Y
    Q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    alpha = np.minimum(proj.opacity[0] * np.exp(-0.5 * Q), st.alpha_max)
    keep = (Q <= st.q_max) & (alpha >= st.alpha_min)
    s, m = orc.scene_importance(sc, [cam], np.ones(1), st)
    assert keep.sum() > 50
    np.testing.assert_allclose(s[0], alpha[keep].sum(), rtol=1e-12)
    np.testing.assert_allclose(m[0], alpha[keep].max(), rtol=1e-12)
