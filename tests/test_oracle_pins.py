"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, special cases that reduce to the
standard blender, invariants, finite differences and an independent dense
autodiff reference (tests/dense_ref.py).  A plausible mistake anywhere in the
oracle (a dropped term, a sign, an index, a transposed operand) fails at least
one of them.
"""
import math

import numpy as np
import pytest
import torch

import scenegen
from tests import dense_ref


def _small(n=32, w=32, h=24, seed=5, deg=2, ls=-1.8, depth=4.0, opacity_mean=0.0, n_views=1):
    return scenegen.small_scene(n, w, h, seed=seed, sh_degree=deg, log_scale_mean=ls, depth=depth,
                                opacity_mean=opacity_mean, n_views=n_views)


# ---------------------------------------------------------------------------
# Philox4x32-10: known-answer vectors published with the generator (Random123)
# ---------------------------------------------------------------------------

def test_philox_known_answers(orc):
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert list(orc.philox4x32_10(ctr, key)) == want


# ---------------------------------------------------------------------------
# spherical harmonics (Sec. 3.1: view-dependent SH colour)
# ---------------------------------------------------------------------------

def test_sh_orthonormal_by_quadrature(orc):
    zs, wz = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phis = 2 * np.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(zs, phis, indexing="ij")
    WZ = np.repeat(wz[:, None], nphi, axis=1) * (2 * np.pi / nphi)
    st = np.sqrt(1 - Z ** 2)
    dirs = np.stack([st * np.cos(PHI), st * np.sin(PHI), Z], -1).reshape(-1, 3)
    Y, _ = orc.sh_basis(3, dirs)
    gram = (Y * WZ.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_low_degree_closed_forms(orc):
    rng = np.random.default_rng(0)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, _ = orc.sh_basis(1, d)
    np.testing.assert_allclose(Y[:, 0], 1.0 / (2.0 * math.sqrt(math.pi)), rtol=1e-15)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    np.testing.assert_allclose(Y[:, 1], c1 * d[:, 1], rtol=1e-14)
    np.testing.assert_allclose(Y[:, 2], c1 * d[:, 2], rtol=1e-14)
    np.testing.assert_allclose(Y[:, 3], c1 * d[:, 0], rtol=1e-14)


def test_sh_matches_cartesian_table_and_gradient(orc):
    rng = np.random.default_rng(1)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, dY = orc.sh_basis(3, d)
    Yc = dense_ref.sh_cartesian(3, torch.tensor(d)).numpy()
    np.testing.assert_allclose(Y, Yc, atol=1e-14)
    # tangential gradient vs central differences along the sphere
    h = 1e-6
    for k in range(16):
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            dp = (d + e) / np.linalg.norm(d + e, axis=1, keepdims=True)
            dm = (d - e) / np.linalg.norm(d - e, axis=1, keepdims=True)
            fd = (orc.sh_basis(3, dp)[0][:, k] - orc.sh_basis(3, dm)[0][:, k]) / (2 * h)
            g = dY[:, k, :]
            # moving v = d along e_j moves dir = v/|v| by e_j - d d_j (|d| = 1)
            an = g[:, j] - d[:, j] * np.sum(g * d, axis=1)
            np.testing.assert_allclose(fd, an, atol=2e-8)


# ---------------------------------------------------------------------------
# projection and a single Gaussian (Sec. 3.1)
# ---------------------------------------------------------------------------

def _one_gaussian_scene(mean, log_scale, quat=(1, 0, 0, 0), opacity_logit=0.0, rgb=(0.8, 0.3, 0.1)):
    y00 = 0.5 / math.sqrt(math.pi)
    return dict(means=np.array([mean], np.float32), log_scales=np.array([[log_scale] * 3], np.float32),
                quats=np.array([quat], np.float32), opacity_logits=np.array([opacity_logit], np.float32),
                sh=((np.array([[rgb]], np.float64) - 0.5) / y00).astype(np.float32))


def test_isotropic_on_axis_projection_closed_form(orc):
    cam = scenegen.orbit_camera(4.0, 0.0, 0.0, 64, 48)
    ls = math.log(0.05)
    sc = _one_gaussian_scene([0.0, 0.0, 0.0], ls, quat=(0.3, -0.5, 0.2, 0.7))
    st = orc.RasterSettings(sh_degree=0)
    pr = orc.project(sc, cam, st)
    s = math.exp(float(np.float32(ls)))
    fx = float(cam["fx"])
    var = (fx * s / 4.0) ** 2 + float(np.float32(0.3))
    np.testing.assert_allclose(pr.cov2d[0], [var, 0.0, var], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pr.conic[0], [1 / var, 0.0, 1 / var], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pr.mean2d[0], [32.0, 24.0], atol=1e-12)
    assert pr.depth[0] == np.float32(4.0)
    # isotropic: the eigenvalue discriminant is 0 and takes its floor 0.1
    assert pr.radius[0] == math.ceil(3 * math.sqrt(var + math.sqrt(float(np.float32(0.1)))))
    np.testing.assert_allclose(pr.color[0], [0.8, 0.3, 0.1], atol=1e-7)


def _clamped_cov2d(cam, t, s, dil):
    """Sigma_2D of an isotropic Gaussian (scale s) at view-space centre t,
    with the lateral ratios of the Jacobian clamped at 1.3 tan(fov / 2):
    J J^T s^2 + dil I written out for J = [[f/z, 0, -f r_x], [0, f/z, -f r_y]]
    / ... with r = clamp(t_xy / z), so (J J^T)_00 = fx^2 (1 + r_x^2) / z^2,
    (J J^T)_01 = fx fy r_x r_y / z^2, (J J^T)_11 = fy^2 (1 + r_y^2) / z^2."""
    fx, fy = float(cam["fx"]), float(cam["fy"])
    limx = float(np.float32(1.3)) * 0.5 * cam["width"] / fx
    limy = float(np.float32(1.3)) * 0.5 * cam["height"] / fy
    rx = min(max(t[0] / t[2], -limx), limx)
    ry = min(max(t[1] / t[2], -limy), limy)
    z2 = t[2] * t[2]
    return np.array([s * s * fx * fx * (1 + rx * rx) / z2 + dil, s * s * fx * fy * rx * ry / z2,
                     s * s * fy * fy * (1 + ry * ry) / z2 + dil]), (abs(t[0] / t[2]) > limx, abs(t[1] / t[2]) > limy)


@pytest.mark.parametrize("t", [(0.3, -0.2, 4.0), (4.8, 0.0, 4.0), (-4.4, 0.0, 4.0), (0.0, -3.6, 4.0),
                               (0.0, 2.9, 4.0), (5.1, -3.3, 4.0), (-2.6, 2.5, 2.5)])
def test_clamped_jacobian_projection_closed_form(orc, t):
    """Sec. 3.1 (EWA splatting): an isotropic Gaussian anywhere in front of
    the camera, inside and beyond the lateral clamp of the Jacobian in x, in
    y and in both, with both signs: Sigma_2D and the conic in closed form."""
    cam = scenegen.orbit_camera(4.0, 0.0, 0.0, 64, 48)  # identity rotation, centre at (0, 0, -4)
    ls = float(np.float32(math.log(0.07)))
    sc = _one_gaussian_scene([t[0], t[1], t[2] - 4.0], ls, quat=(0.6, 0.1, -0.7, 0.2))
    st = orc.RasterSettings(sh_degree=0)
    pr = orc.project(sc, cam, st)
    tt = np.array(sc["means"][0], np.float64) + np.array([0.0, 0.0, 4.0])
    want, (cx, cy) = _clamped_cov2d(cam, tt, math.exp(ls), float(np.float32(0.3)))
    np.testing.assert_allclose(pr.cov2d[0], want, rtol=1e-12, atol=1e-12 * want.max())
    det = want[0] * want[2] - want[1] ** 2
    wc = np.array([want[2] / det, -want[1] / det, want[0] / det])
    np.testing.assert_allclose(pr.conic[0], wc, rtol=1e-11, atol=1e-12 * np.abs(wc).max())
    fx = float(cam["fx"])
    np.testing.assert_allclose(pr.mean2d[0], [fx * tt[0] / tt[2] + 32.0, fx * tt[1] / tt[2] + 24.0], rtol=1e-13)
    if abs(t[0]) > 4 or abs(t[1]) > 3:
        assert cx or cy  # the case reaches the clamp


def test_clamped_jacobian_finite_differences(orc):
    """O10 through the clamped branch of the Jacobian: central differences in
    exact mode of every continuous input of splats beyond the clamp in x, in
    y, in both (either sign) and inside it, whose footprints reach into the
    image; the clamped ratio has zero derivative in the view-space centre."""
    cam = scenegen.orbit_camera(4.0, 0.0, 0.0, 24, 18)
    fx = float(cam["fx"])
    limx, limy = 1.3 * 12 / fx, 1.3 * 9 / fx
    ts = [(1.25 * limx, 0.1, 1.0), (-1.3 * limx, -0.05, 1.0), (0.05, 1.3 * limy, 1.0), (-0.1, -1.35 * limy, 1.0),
          (1.2 * limx, -1.25 * limy, 1.0), (0.1, 0.1, 1.0)]
    rng = np.random.default_rng(12)
    n = len(ts)
    # distinct depths (4 + 0.3 k), so that no difference reorders the splats
    means = np.array([[r * (4.0 + 0.3 * k), q * (4.0 + 0.3 * k), 0.3 * k] for k, (r, q, _) in enumerate(ts)])
    sc = dict(means=means.astype(np.float32),
              log_scales=(np.log(0.9) + 0.2 * rng.normal(size=(n, 3))).astype(np.float32),
              quats=rng.normal(size=(n, 4)).astype(np.float32),
              opacity_logits=rng.normal(size=n).astype(np.float32),
              sh=(0.4 * rng.normal(size=(n, 4, 3))).astype(np.float32))
    clamped = 0
    for r, q, _ in ts:
        clamped += (abs(r) > limx) + (abs(q) > limy)
    assert clamped >= 6
    st = orc.RasterSettings(sh_degree=1, bg=(0.2, 0.5, 0.1), exact_mode=True)
    mask = rng.uniform(0.3, 1.0, n)
    P = 24 * 18
    w = rng.normal(size=3 * P)
    base = {k: np.asarray(sc[k], np.float64).copy() for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    out = orc.run_pipeline(base, [cam], mask, st, dl_dimage=w)
    assert np.all(out.proj[0].valid == 1)
    grads = dict(means=out.grads.means, log_scales=out.grads.log_scales, quats=out.grads.quats)
    h = 1e-6
    for key, g in grads.items():
        flat = base[key].reshape(-1)
        fd = np.zeros(flat.size)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp = _loss_linear(orc, base, [cam], mask, st, w)
            flat[j] = old - h
            lm = _loss_linear(orc, base, [cam], mask, st, w)
            flat[j] = old
            fd[j] = (lp - lm) / (2 * h)
        scale = max(np.abs(fd).max(), 1e-3)
        assert np.abs(fd - g.reshape(-1)).max() <= 2e-6 * scale, (key, np.abs(fd - g.reshape(-1)).max() / scale)
        # every splat's gradient is resolved (the footprints reach the image)
        assert np.all(np.abs(fd.reshape(n, -1)).max(axis=1) > 1e-6 * scale), key


def _flag_case(orc, mean2d, opacity, depth_bits, w=1, h=1, st=None):
    """Flags and final transmittance of pixel (0, 0) of a one-pixel image for
    splats given by their 2D centres (conic = identity), opacities and depth
    bits."""
    st = st or orc.RasterSettings(sh_degree=0)
    n = len(opacity)
    m2 = np.asarray(mean2d, np.float64).reshape(n, 2)
    conic = np.tile([1.0, 0.0, 1.0], (n, 1))
    rad = np.full(n, 20.0)
    lists = orc.build_lists([w], [h], n, m2, rad, np.asarray(depth_bits, np.uint32), np.ones(n, np.uint8), st)
    col = np.tile([0.5, 0.25, 0.75], (n, 1))
    of = orc.render_fwd([w], [h], n, m2, conic, np.asarray(opacity, np.float64), col, np.ones(n), lists, st)
    ob = orc.render_bwd([w], [h], n, m2, conic, np.asarray(opacity, np.float64), col, np.ones(n), lists,
                        np.ones(3 * w * h), st)
    return int(of.flags[0]), of, ob


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_decision_flags_mark_only_near_threshold_cases(orc, sign):
    """The parity protocol's decision margins: a pixel is flagged when a
    discrete decision of its walk lies within a relative 1e-5 of its
    threshold (Q vs 9, o G vs 0.99, alpha vs 1/255) or 2e-4 (the stop test
    vs T_min), and only then; flagged pixels mark every entry they touch."""
    FQ, FAMIN, FAMAX, FT = 1, 2, 4, 8
    pc = 0.5  # centre of pixel (0, 0)
    # Q = d^2 for a splat at distance d with the identity conic
    for eps, flagged in [(5e-6, True), (1e-3, False)]:
        d = 3.0 * math.sqrt(1.0 + sign * eps)
        f, _, _ = _flag_case(orc, [[pc + d, pc]], [0.9], [1])
        assert bool(f & FQ) == flagged, (eps, f)
        # alpha against the filter 1/255 (Q = 0: alpha = opacity)
        a = float(np.float32(1 / 255)) * (1.0 + sign * eps)
        f, _, _ = _flag_case(orc, [[pc, pc]], [a], [1])
        assert bool(f & FAMIN) == flagged, (eps, f)
        # o G against the clamp 0.99
        f, _, _ = _flag_case(orc, [[pc, pc]], [0.99 * (1.0 + sign * eps)], [1])
        assert bool(f & FAMAX) == flagged, (eps, f)
    # the stop test T (1 - alpha) against T_min = 1e-4 after two splats of 0.95
    for eps, flagged in [(1e-4, True), (1e-2, False)]:
        a3 = 1.0 - 0.04 * (1.0 + sign * eps)
        f, of, ob = _flag_case(orc, [[pc, pc]] * 4, [0.95, 0.95, a3, 0.5], [1, 2, 3, 4])
        assert bool(f & FT) == flagged, (eps, f)
        assert f & ~FT == 0
        if flagged:
            # a flagged stop marks the entries up to the stop and those a
            # non-stopping walk would blend next
            assert np.all(ob.touched_flagged[:4] == 1)
        else:
            assert np.all(ob.touched_flagged == 0)
    # far from every threshold: nothing flagged
    f, _, ob = _flag_case(orc, [[pc + 1.0, pc], [pc, pc + 2.0]], [0.5, 0.7], [1, 2])
    assert f == 0 and np.all(ob.touched_flagged == 0)


@pytest.mark.parametrize("mval", [1.0, 0.0, 0.37])
def test_single_gaussian_image_closed_form(orc, mval):
    cam = scenegen.orbit_camera(4.0, 0.0, 0.0, 40, 36)
    sc = _one_gaussian_scene([0.05, -0.03, 0.1], math.log(0.06), opacity_logit=1.2)
    bg = (0.1, 0.5, 0.9)
    st = orc.RasterSettings(sh_degree=0, bg=bg)
    out = orc.run_pipeline(sc, [cam], np.array([mval]), st, backward=False)
    pr = out.proj[0]
    H, W = 36, 40
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    dx, dy = pr.mean2d[0, 0] - xs, pr.mean2d[0, 1] - ys
    a, b, c = pr.conic[0]
    Q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    al = np.minimum(0.99, pr.opacity[0] * np.exp(-Q / 2))
    keep = (Q <= 9) & (al >= np.float32(1 / 255))
    al = np.where(keep, al, 0.0)
    want = np.stack([mval * pr.color[0, ch] * al + (1 - mval * al) * np.float32(bg[ch]) for ch in range(3)])
    np.testing.assert_allclose(out.fwd.image.reshape(3, H, W), want, rtol=0, atol=1e-14)
    # symmetry: an on-axis isotropic Gaussian in a square image is mirror-symmetric
    sc2 = _one_gaussian_scene([0.0, 0.0, 0.0], math.log(0.1), opacity_logit=0.5)
    cam2 = scenegen.orbit_camera(4.0, 0.0, 0.0, 32, 32)
    im = orc.run_pipeline(sc2, [cam2], np.array([mval]), st, backward=False).fwd.image.reshape(3, 32, 32)
    np.testing.assert_allclose(im, im[:, ::-1, :], atol=1e-14)
    np.testing.assert_allclose(im, im[:, :, ::-1], atol=1e-14)


# ---------------------------------------------------------------------------
# special cases of masked compositing, Eq. (3)-(4)
# ---------------------------------------------------------------------------

def _standard_blend(out, n, mask_unused, st, w, h):
    """Eq. (1)-(2) without masks, walking the oracle's own tile lists."""
    pr = out.proj[0]
    img = np.zeros((3, h, w))
    tfin = np.zeros((h, w))
    gw = (w + st.tile_w - 1) // st.tile_w
    for y in range(h):
        for x in range(w):
            t = (y // st.tile_h) * gw + x // st.tile_w
            s, e = out.lists.ranges[t]
            T = 1.0
            C = np.zeros(3)
            for k in range(s, e):
                g = out.lists.vals[k]
                dx, dy = pr.mean2d[g, 0] - (x + 0.5), pr.mean2d[g, 1] - (y + 0.5)
                a, b, c = pr.conic[g]
                Q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
                if Q > st.q_max:
                    continue
                alpha = min(float(np.float32(st.alpha_max)), pr.opacity[g] * math.exp(-0.5 * Q))
                if alpha < float(np.float32(st.alpha_min)):
                    continue
                if T * (1.0 - alpha) < float(np.float32(st.t_min)):
                    break
                C += alpha * T * pr.color[g]
                T = T * (1.0 - alpha)
            img[:, y, x] = C + T * np.array([float(np.float32(b_)) for b_ in st.bg])
            tfin[y, x] = T
    return img, tfin


def test_all_ones_masks_equal_standard_blending(orc):
    sc = _small(n=40, w=24, h=20, seed=11, deg=1, ls=-2.0)
    st = orc.RasterSettings(sh_degree=1, bg=(0.2, 0.4, 0.1))
    cam = sc["cameras"][0]
    out = orc.run_pipeline(sc, [cam], np.ones(40), st, backward=False)
    img, tfin = _standard_blend(out, 40, None, st, 24, 20)
    np.testing.assert_allclose(out.fwd.image.reshape(3, 20, 24), img, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out.fwd.t_final.reshape(20, 24), tfin, rtol=0, atol=1e-15)


def test_all_zero_masks_give_background_and_closed_form_mask_grad(orc):
    sc = _small(n=48, w=32, h=24, seed=12, deg=2, ls=-1.8)
    bg = (0.3, 0.6, 0.2)
    st = orc.RasterSettings(sh_degree=2, bg=bg)
    cam = sc["cameras"][0]
    rng = np.random.default_rng(2)
    w = rng.normal(size=3 * 32 * 24)
    out = orc.run_pipeline(sc, [cam], np.zeros(48), st, dl_dimage=w)
    bgv = np.array([float(np.float32(b)) for b in bg])
    assert np.array_equal(out.fwd.image.reshape(3, -1), np.repeat(bgv[:, None], 32 * 24, axis=1))
    assert np.all(out.fwd.t_final == 1.0)
    for arr in (out.bwd.d_mean2d, out.bwd.d_conic, out.bwd.d_opacity, out.bwd.d_color):
        assert np.all(arr == 0.0)
    for arr in (out.grads.means, out.grads.log_scales, out.grads.quats, out.grads.opacity_logits, out.grads.sh):
        assert np.all(arr == 0.0)
    # dL/dM_i = sum over pixels of alpha_i(px) <w, c_i - bg> (T_i = 1, nothing behind)
    pr = out.proj[0]
    ys, xs = np.mgrid[0:24, 0:32] + 0.5
    W3 = w.reshape(3, 24, 32)
    want = np.zeros(48)
    for g in range(48):
        if not pr.valid[g]:
            continue
        dx, dy = pr.mean2d[g, 0] - xs, pr.mean2d[g, 1] - ys
        a, b, c = pr.conic[g]
        Q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        al = np.minimum(0.99, pr.opacity[g] * np.exp(-Q / 2))
        al = np.where((Q <= 9) & (al >= np.float32(1 / 255)), al, 0.0)
        want[g] = np.sum(al * np.tensordot(pr.color[g] - bgv, W3, axes=(0, 0)))
    np.testing.assert_allclose(out.bwd.d_mask, want, rtol=1e-12, atol=1e-13)


def _loss_linear(orc, sc, cams, mask, st, w):
    out = orc.run_pipeline(sc, cams, mask, st, backward=False)
    return float(np.dot(out.fwd.image, w))


@pytest.mark.parametrize("fractional", [False, True])
def test_flip_identity_mask_gradient(orc, fractional):
    """C is affine in each M_i, so dL/dM_i = L(M_i=1) - L(M_i=0) exactly for a linear L."""
    sc = _small(n=24, w=24, h=20, seed=13, deg=1, ls=-1.7)
    st = orc.RasterSettings(sh_degree=1, bg=(0.5, 0.1, 0.7), exact_mode=True)
    cam = sc["cameras"][0]
    rng = np.random.default_rng(4)
    mask = rng.uniform(0, 1, 24) if fractional else sc["masks"].astype(np.float64)
    w = rng.normal(size=3 * 24 * 20)
    out = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w)
    for i in range(24):
        m1, m0 = mask.copy(), mask.copy()
        m1[i], m0[i] = 1.0, 0.0
        want = _loss_linear(orc, sc, [cam], m1, st, w) - _loss_linear(orc, sc, [cam], m0, st, w)
        assert abs(out.bwd.d_mask[i] - want) <= 1e-10 * max(1.0, abs(want))


def test_mask_opacity_identity(orc):
    """For M_i = 1 and no clamped alpha, dL/dM_i = o_i dL/do_i (alpha = o G)."""
    sc = _small(n=40, w=32, h=24, seed=14, deg=2, ls=-1.8, opacity_mean=-1.0)
    st = orc.RasterSettings(sh_degree=2, bg=(0.2, 0.2, 0.9))
    cam = sc["cameras"][0]
    rng = np.random.default_rng(5)
    w = rng.normal(size=3 * 32 * 24)
    mask = np.ones(40)
    mask[::3] = 0.0
    out = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=w)
    o = out.proj[0].opacity
    assert np.all(o < 0.99)
    on = mask == 1
    np.testing.assert_allclose(out.bwd.d_mask[on], o[on] * out.bwd.d_opacity[on], rtol=1e-12, atol=1e-14)


def test_fig1_five_gaussians_two_masked(orc):
    """Fig. 1 structure: five splats at one pixel, G2 and G5 masked.

    A 1x1 image whose pixel centre lies on the optical axis; every Gaussian is
    on the axis, so G = 1 and alpha_i = o_i.  Expected values are expanded by
    hand from Eq. (3)-(4), Eq. (6) and the background term.
    """
    cam = scenegen.camera_from_pose(np.eye(3), np.zeros(3), 1, 1)
    depths = [2.0, 3.0, 4.0, 5.0, 6.0]
    logits = [0.2, -0.4, 0.9, -0.1, 0.5]
    rgbs = [(0.9, 0.1, 0.2), (0.2, 0.8, 0.3), (0.1, 0.2, 0.7), (0.6, 0.6, 0.1), (0.3, 0.3, 0.9)]
    y00 = 0.5 / math.sqrt(math.pi)
    sc = dict(means=np.array([[0, 0, d] for d in depths], np.float32),
              log_scales=np.full((5, 3), math.log(0.01), np.float32),
              quats=np.tile(np.array([1, 0, 0, 0], np.float32), (5, 1)),
              opacity_logits=np.array(logits, np.float32),
              sh=((np.array(rgbs)[:, None, :] - 0.5) / y00).astype(np.float32))
    bg = np.array([0.25, 0.5, 0.75])
    st = orc.RasterSettings(sh_degree=0, bg=tuple(bg))
    bg = np.array([float(np.float32(b)) for b in bg])
    M = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    w = np.array([0.7, -1.1, 0.4])
    out = orc.run_pipeline(sc, [cam], M, st, dl_dimage=w)
    o = 1.0 / (1.0 + np.exp(-np.array(logits, np.float32).astype(np.float64)))
    c = out.proj[0].color
    np.testing.assert_allclose(c, np.array(rgbs), atol=1e-7)
    o1, o2, o3, o4, o5 = o
    c1, c2, c3, c4, c5 = c
    T_final = (1 - o1) * (1 - o3) * (1 - o4)
    C = o1 * c1 + (1 - o1) * o3 * c3 + (1 - o1) * (1 - o3) * o4 * c4 + T_final * bg
    np.testing.assert_allclose(out.fwd.image, C, rtol=0, atol=1e-15)
    assert abs(out.fwd.t_final[0] - T_final) < 1e-15
    # colour behind each entry, relative to the transmittance just after it
    b3 = o3 * c3 + (1 - o3) * o4 * c4
    dM2 = o2 * (1 - o1) * np.dot(w, c2 - b3) - o2 * T_final * np.dot(w, bg)
    dM5 = o5 * T_final * np.dot(w, c5) - o5 * T_final * np.dot(w, bg)
    b2 = b3  # G2 is masked: nothing of it behind G1
    dM1 = o1 * np.dot(w, c1 - b2) - o1 * T_final / (1 - o1) * np.dot(w, bg)
    np.testing.assert_allclose(out.bwd.d_mask[[0, 1, 4]], [dM1, dM2, dM5], rtol=1e-13)
    # masked splats get a mask gradient but no colour or opacity gradient
    assert np.all(out.bwd.d_color[[1, 4]] == 0.0) and np.all(out.bwd.d_opacity[[1, 4]] == 0.0)
    assert np.all(out.bwd.d_color[[0, 2, 3]] != 0.0)


# ---------------------------------------------------------------------------
# finite differences and the dense reference
# ---------------------------------------------------------------------------

def test_finite_differences_exact_mode(orc):
    sc = _small(n=6, w=20, h=16, seed=21, deg=2, ls=-1.6, depth=3.5, opacity_mean=-0.5)
    st = orc.RasterSettings(sh_degree=2, bg=(0.4, 0.3, 0.8), exact_mode=True)
    cams = [sc["cameras"][0], scenegen.orbit_camera(3.2, 20.0, 10.0, 18, 14)]
    rng = np.random.default_rng(6)
    mask = rng.uniform(0.2, 1.0, 6)
    P = 20 * 16 + 18 * 14
    w = rng.normal(size=3 * P)
    base = {k: np.asarray(sc[k], np.float64).copy() for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    out = orc.run_pipeline(base, cams, mask, st, dl_dimage=w)
    grads = dict(means=out.grads.means, log_scales=out.grads.log_scales, quats=out.grads.quats,
                 opacity_logits=out.grads.opacity_logits, sh=out.grads.sh)
    h = 1e-6
    for key, g in grads.items():
        flat = base[key].reshape(-1)
        fd = np.zeros(flat.size)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp = _loss_linear(orc, base, cams, mask, st, w)
            flat[j] = old - h
            lm = _loss_linear(orc, base, cams, mask, st, w)
            flat[j] = old
            fd[j] = (lp - lm) / (2 * h)
        scale = max(np.abs(fd).max(), 1e-3)
        assert np.abs(fd - g.reshape(-1)).max() <= 2e-6 * scale, key
    # mask, by central differences too
    fdm = np.zeros(6)
    for j in range(6):
        mp, mm = mask.copy(), mask.copy()
        mp[j] += h
        mm[j] -= h
        fdm[j] = (_loss_linear(orc, base, cams, mp, st, w) - _loss_linear(orc, base, cams, mm, st, w)) / (2 * h)
    np.testing.assert_allclose(out.bwd.d_mask, fdm, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("exact", [False, True])
def test_dense_autodiff_reference(orc, exact):
    sc = _small(n=48, w=40, h=32, seed=7, deg=3, ls=-1.7)
    st = orc.RasterSettings(sh_degree=3, bg=(0.3, 0.2, 0.6), exact_mode=exact)
    cam = sc["cameras"][0]
    m = sc["masks"].astype(np.float64)
    rng = np.random.default_rng(3)
    w = rng.normal(size=3 * 40 * 32)
    out = orc.run_pipeline(sc, [cam], m, st, dl_dimage=w)
    p = dense_ref.params_from_scene(sc)
    mt = torch.tensor(m, requires_grad=True)
    C, T = dense_ref.render_dense(p, cam, st, mt)
    np.testing.assert_allclose(out.fwd.image.reshape(3, 32, 40), C.detach().numpy(), atol=1e-13)
    np.testing.assert_allclose(out.fwd.t_final.reshape(32, 40), T.detach().numpy(), atol=1e-13)
    (C.reshape(-1) * torch.tensor(w)).sum().backward()
    pairs = [(out.grads.means, p["means"].grad), (out.grads.log_scales, p["log_scales"].grad),
             (out.grads.quats, p["quats"].grad), (out.grads.opacity_logits, p["opacity_logits"].grad),
             (out.grads.sh, p["sh"].grad), (out.bwd.d_mask, mt.grad)]
    for a, b in pairs:
        b = b.numpy()
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())


# ---------------------------------------------------------------------------
# tile lists, order and invariances (Sec. 3.1)
# ---------------------------------------------------------------------------

def test_list_properties_and_coverage(orc):
    sc = _small(n=64, w=48, h=40, seed=31, deg=0, ls=-2.2)
    st = orc.RasterSettings(sh_degree=0)
    cam = sc["cameras"][0]
    out = orc.run_pipeline(sc, [cam], sc["masks"], st, backward=False)
    L = out.lists
    assert L.keys.size == int(L.tiles_touched.sum())
    # lexicographic (key, value) order
    order = np.lexsort((L.vals, L.keys))
    assert np.array_equal(order, np.arange(L.keys.size))
    tiles = (L.keys >> np.uint64(32)).astype(np.int64)
    for t in range(L.total_tiles):
        s, e = L.ranges[t]
        assert np.all(tiles[s:e] == t)
    # every (pixel, Gaussian) pair with Q <= 9 at the pixel is in that pixel's tile list
    pr = out.proj[0]
    gw = 3
    for y in range(40):
        for x in range(48):
            t = (y // 16) * gw + x // 16
            s, e = L.ranges[t]
            members = set(L.vals[s:e].tolist())
            for g in range(64):
                if not pr.valid[g]:
                    continue
                dx, dy = pr.mean2d[g, 0] - (x + 0.5), pr.mean2d[g, 1] - (y + 0.5)
                a, b, c = pr.conic[g]
                if a * dx * dx + 2 * b * dx * dy + c * dy * dy <= 9.0:
                    assert g in members


def test_tile_size_invariance(orc):
    sc = _small(n=80, w=50, h=36, seed=41, deg=1, ls=-1.9)
    cam = sc["cameras"][0]
    ref = None
    for tw, th in [(16, 16), (8, 8), (16, 8), (32, 8)]:
        st = orc.RasterSettings(sh_degree=1, tile_w=tw, tile_h=th, bg=(0.1, 0.2, 0.3))
        out = orc.run_pipeline(sc, [cam], sc["masks"], st, backward=False)
        if ref is None:
            ref = out.fwd
        else:
            assert np.array_equal(out.fwd.image, ref.image)
            assert np.array_equal(out.fwd.t_final, ref.t_final)
            assert np.array_equal(out.fwd.n_blend, ref.n_blend)


def test_permutation_invariance(orc):
    sc = _small(n=60, w=40, h=30, seed=42, deg=1, ls=-1.9)
    st = orc.RasterSettings(sh_degree=1, bg=(0.2, 0.1, 0.3))
    cam = sc["cameras"][0]
    rng = np.random.default_rng(8)
    w = rng.normal(size=3 * 40 * 30)
    perm = rng.permutation(60)
    sc2 = {k: (np.asarray(v)[perm] if isinstance(v, np.ndarray) and v.shape[:1] == (60,) else v)
           for k, v in sc.items()}
    a = orc.run_pipeline(sc, [cam], sc["masks"], st, dl_dimage=w)
    b = orc.run_pipeline(sc2, [cam], sc2["masks"], st, dl_dimage=w)
    assert len(set(a.proj[0].depth_bits.tolist())) == 60
    np.testing.assert_allclose(a.fwd.image, b.fwd.image, rtol=0, atol=1e-15)
    np.testing.assert_allclose(a.bwd.d_mask[perm], b.bwd.d_mask, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(a.grads.means[perm], b.grads.means, rtol=1e-12, atol=1e-14)
    # Gaussian j of the permuted scene is Gaussian perm[j] of the original
    assert np.array_equal(perm[b.lists.vals], a.lists.vals)


def test_direct_pixels_equal_tiled(orc):
    sc = _small(n=120, w=64, h=48, seed=51, deg=2, ls=-2.0)
    st = orc.RasterSettings(sh_degree=2, bg=(0.3, 0.3, 0.3))
    cam = sc["cameras"][0]
    out = orc.run_pipeline(sc, [cam], sc["masks"], st, backward=False)
    rng = np.random.default_rng(9)
    px = np.stack([rng.integers(0, 64, 200), rng.integers(0, 48, 200)], 1)
    rgb, tf, nb = orc.render_pixels_direct(out.proj[0], sc["masks"], px, st)
    img = out.fwd.image.reshape(3, 48, 64)
    np.testing.assert_allclose(rgb, img[:, px[:, 1], px[:, 0]].T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tf, out.fwd.t_final.reshape(48, 64)[px[:, 1], px[:, 0]], rtol=0, atol=1e-15)
    assert np.array_equal(nb, out.fwd.n_blend.reshape(48, 64)[px[:, 1], px[:, 0]])


def test_multiview_equals_separate_views(orc):
    sc = _small(n=50, w=30, h=20, seed=61, deg=1, ls=-1.9, n_views=3)
    cams = sc["cameras"]
    cams[1] = scenegen.orbit_camera(4.0, 40.0, 5.0, 22, 26)
    st = orc.RasterSettings(sh_degree=1, bg=(0.1, 0.6, 0.2))
    rng = np.random.default_rng(10)
    P = sum(c["width"] * c["height"] for c in cams)
    w = rng.normal(size=3 * P)
    allv = orc.run_pipeline(sc, cams, sc["masks"], st, dl_dimage=w)
    off = 0
    gsum = np.zeros_like(allv.grads.means)
    dm = np.zeros(50)
    for c in cams:
        p = c["width"] * c["height"]
        one = orc.run_pipeline(sc, [c], sc["masks"], st, dl_dimage=w[3 * off:3 * (off + p)])
        np.testing.assert_array_equal(allv.fwd.image[3 * off:3 * (off + p)], one.fwd.image)
        gsum += one.grads.means
        dm += one.bwd.d_mask
        off += p
    np.testing.assert_allclose(allv.grads.means, gsum, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(allv.bwd.d_mask, dm, rtol=1e-12, atol=1e-14)


def test_early_stop_excludes_stop_entry(orc):
    """Opaque stack at one pixel: T after k entries is prod(1 - o); the entry
    that would take T below T_min is excluded and gets no gradient."""
    cam = scenegen.camera_from_pose(np.eye(3), np.zeros(3), 1, 1)
    n = 6
    y00 = 0.5 / math.sqrt(math.pi)
    sc = dict(means=np.array([[0, 0, 2.0 + k] for k in range(n)], np.float32),
              log_scales=np.full((n, 3), math.log(0.01), np.float32),
              quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
              opacity_logits=np.full(n, 4.0, np.float32),
              sh=np.full((n, 1, 3), (0.7 - 0.5) / y00, np.float32))
    st = orc.RasterSettings(sh_degree=0)
    mask = np.ones(n)
    mask[1] = 0.0
    out = orc.run_pipeline(sc, [cam], mask, st, dl_dimage=np.ones(3))
    o = 1 / (1 + np.exp(-np.float32(4.0).astype(np.float64)))
    # T: 1, (1-o) after G0, unchanged by masked G1, then (1-o)^2 ... stop when < 1e-4
    T = 1.0
    kept = []
    for k in range(n):
        t2 = T * (1 - mask[k] * o)
        if t2 < np.float32(1e-4):
            break
        kept.append(k)
        T = t2
    assert out.fwd.n_blend[0] == len(kept)
    assert abs(out.fwd.t_final[0] - T) < 1e-15
    assert np.all(out.bwd.d_mask[len(kept):] == 0.0)
    assert out.bwd.d_mask[1] != 0.0


# ---------------------------------------------------------------------------
# masks: Gumbel-Softmax sampling and the mask loss (Sec. 3.3, Eq. 7-8)
# ---------------------------------------------------------------------------

def test_gumbel_frequency_matches_sigmoid(orc):
    n = 200_000
    for ell in (-1.5, 0.0, 0.8, 2.5):
        scores = np.zeros((n, 2), np.float32)
        scores[:, 0] = ell
        hits = 0
        for step in range(5):
            m, _ = orc.sample_masks(scores, 0.5, seed=1234, step=step)
            hits += m.sum()
        p = 1 / (1 + math.exp(-float(np.float32(ell))))
        N = 5 * n
        assert abs(hits / N - p) <= 5 * math.sqrt(p * (1 - p) / N)


def test_prune_keep_rate_matches_closed_form(orc):
    """Sec. 3.5: a Gaussian survives unless all n_draws independent hard draws
    are 0, so P(keep) = 1 - (1 - sigmoid(s0 - s1))^n_draws; checked within a
    5-sigma binomial bound, with the draws' independence across steps implied."""
    n = 200_000
    for ell, draws in ((-3.0, 10), (-1.0, 10), (0.5, 3), (-2.0, 1)):
        scores = np.zeros((n, 2), np.float32)
        scores[:, 0] = ell
        keep = orc.prune_keep(scores, seed=77, step0=1000, n_draws=draws)
        p = 1 / (1 + math.exp(-float(np.float32(ell))))
        q = 1 - (1 - p) ** draws
        assert abs(keep.mean() - q) <= 5 * math.sqrt(q * (1 - q) / n)


def test_prune_keep_limits_and_single_draw(orc):
    """A Gaussian whose "exists" score dominates by far is always kept, one
    dominated by far never; with one draw, keep equals that step's hard mask."""
    scores = np.zeros((1000, 2), np.float32)
    scores[:500, 0] = 60.0
    scores[500:, 1] = 60.0
    keep = orc.prune_keep(scores, seed=5, step0=0, n_draws=10)
    assert keep[:500].all() and not keep[500:].any()
    rng = np.random.default_rng(4)
    sc = rng.normal(size=(5000, 2)).astype(np.float32)
    m, _ = orc.sample_masks(sc, 0.5, seed=9, step=42)
    assert np.array_equal(orc.prune_keep(sc, seed=9, step0=42, n_draws=1), m > 0.5)


def test_gumbel_noise_is_standard_gumbel(orc):
    scores = np.zeros((400_000, 2), np.float32)
    _, _, g = orc.sample_masks(scores, 1.0, seed=99, step=3, return_noise=True)
    g = g.reshape(-1)
    euler_gamma = 0.5772156649015329
    assert abs(g.mean() - euler_gamma) < 5 * (math.pi / math.sqrt(6)) / math.sqrt(g.size)
    assert abs(g.var() - math.pi ** 2 / 6) < 0.02
    # the two noises of one Gaussian and of neighbouring Gaussians are uncorrelated
    G = g.reshape(-1, 2)
    assert abs(np.corrcoef(G[:, 0], G[:, 1])[0, 1]) < 0.01
    assert abs(np.corrcoef(G[:-1, 0], G[1:, 0])[0, 1]) < 0.01


def test_gumbel_soft_sample_limits_and_st_gradient(orc):
    rng = np.random.default_rng(11)
    scores = rng.normal(size=(1000, 2)).astype(np.float32)
    m, y, g = orc.sample_masks(scores, 0.5, seed=7, step=2, return_noise=True)
    z = scores.astype(np.float64) + g
    assert np.array_equal(m, (z[:, 0] > z[:, 1]).astype(np.float64))
    _, y_cold = orc.sample_masks(scores, 1e-6, seed=7, step=2)
    far = np.abs(z[:, 0] - z[:, 1]) > 1e-4
    assert np.array_equal(np.round(y_cold[far]), m[far])
    # straight-through: dL/ds0 = dL/dM * dy/ds0; check dy/ds0 by differences
    tau = 0.5
    dM = rng.normal(size=1000)
    d, _ = orc.mask_grad(dM, m, y, tau, lambda_m=0.0)
    h = 1e-6
    yp = 1 / (1 + np.exp(-((z[:, 0] + h) - z[:, 1]) / tau))
    ym = 1 / (1 + np.exp(-((z[:, 0] - h) - z[:, 1]) / tau))
    np.testing.assert_allclose(d[:, 0], dM * (yp - ym) / (2 * h), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(d[:, 1], -d[:, 0], rtol=0, atol=0)


def test_mask_loss_gradient(orc):
    rng = np.random.default_rng(12)
    n = 50
    m = (rng.uniform(size=n) < 0.6).astype(np.float64)
    y = rng.uniform(0.05, 0.95, n)
    tau, lam = 0.7, 0.3
    d, lm = orc.mask_grad(np.zeros(n), m, y, tau, lam)
    assert abs(lm - (m.mean()) ** 2) < 1e-15
    # d L_m / d M_i by central differences of (mean M)^2 at the hard values
    h = 1e-6
    for i in range(5):
        mp, mm = m.copy(), m.copy()
        mp[i] += h
        mm[i] -= h
        fd = (mp.mean() ** 2 - mm.mean() ** 2) / (2 * h)
        want = lam * fd * y[i] * (1 - y[i]) / tau
        assert abs(d[i, 0] - want) < 1e-9 * max(1, abs(want))


# ---------------------------------------------------------------------------
# losses and optimiser
# ---------------------------------------------------------------------------

def test_l1_loss_and_psnr(orc):
    img = np.array([0.5, 0.2, 0.9, 0.4])
    tgt = np.array([0.5, 0.4, 0.6, 0.1], np.float32)
    loss, d = orc.l1_loss(img, tgt)
    t64 = tgt.astype(np.float64)
    assert abs(loss - np.abs(img - t64).mean()) < 1e-16
    np.testing.assert_array_equal(d, np.array([0.0, -0.25, 0.25, 0.25]))
    assert abs(orc.psnr(np.zeros(4), np.full(4, 0.1)) - 20.0) < 1e-12


def test_adam_two_steps_closed_form(orc):
    g1, g2 = np.array([0.3, -2.0, 1e-3]), np.array([0.1, 1.0, -1e-3])
    p = np.array([1.0, 2.0, 3.0])
    m1, m2 = np.zeros(3), np.zeros(3)
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-15
    orc.adam(p, g1.copy(), m1, m2, lr, b1, b2, eps, 1)
    # first step: m_hat = g, v_hat = g^2, so the step is lr * sign(g)
    np.testing.assert_allclose(p, [1.0 - lr, 2.0 + lr, 3.0 - lr], rtol=1e-12)
    orc.adam(p, g2.copy(), m1, m2, lr, b1, b2, eps, 2)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(p, np.array([1.0 - lr, 2.0 + lr, 3.0 - lr]) - lr * mh / np.sqrt(vh), rtol=1e-12)
