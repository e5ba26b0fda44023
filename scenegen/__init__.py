"""Seeded synthetic scenes and cameras for masked Gaussian rasterization.

This module is shared by the GPU path's tests/benchmark and by the CPU oracle's
tests.  It only draws random numbers and lays them out; it holds none of the
rasterization arithmetic (no projection, no compositing, no gradients).

Every draw uses numpy's PCG64 with seed ``SEED_BASE + config_number`` and the
draw order written in each generator's docstring, so two runs produce
byte-identical arrays.

Layouts (all float32, C-contiguous, N = number of Gaussians):
  means          [N, 3]   world-space centres
  log_scales     [N, 3]   per-axis log standard deviations
  quats          [N, 4]   rotation quaternion (w, x, y, z), unit length
  opacity_logits [N]      opacity = sigmoid(logit)
  sh             [N, (d+1)^2, 3]  real spherical-harmonic coefficients,
                          coefficient-major, index l*l + l + m
  mask_scores    [N, 2]   two existence scores per Gaussian (column 0 =
                          "exists"); P(M = 1) = sigmoid(s0 - s1)
  masks          [N]      a sampled hard mask in {0, 1} (configs that draw
                          Bernoulli masks once)

Cameras are dicts with ``viewmat`` (4x4 float32, world->camera, row-major,
camera +z forward, +y down, +x right), ``fx, fy, cx, cy`` and ``width,
height``.  Every camera has a 60 degree horizontal field of view,
``cx = W/2`` and ``cy = H/2``.

The paper's scenes (Mip-NeRF360, Tanks&Temples, Deep Blending; 0.33-5.81 M
Gaussians, Tables 12-13) are not available; these draws stand in for them with
the Gaussian counts, SH degree and scale statistics of such scenes.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2412_20522_0

# The degree-0 real spherical harmonic is the constant 1/(2 sqrt(pi)); a DC
# coefficient (rgb - 0.5) / Y00 therefore yields base colour rgb once the
# renderer adds its +0.5 offset.  Used only to lay out colour inputs.
_Y00 = 0.5 / math.sqrt(math.pi)

# Largest per-axis log-scale drawn from the heavy-tailed Student-t recipe.
# The 2D covariance of a splat, its determinant a c - b^2, the conic and the
# chain rule back to the scales are evaluated in double precision by the
# oracle and by the GPU alike, and keep about 16 - log10(lambda_max /
# lambda_min) significant digits (the smaller eigenvalue is at least the
# 0.3 px^2 dilation).  A 50-unit axis seen from the nearest depths of these
# cameras reaches an eigenvalue ratio of about 1e11, where the FP64 result is
# still good to the parity tolerances; much longer axes (the uncapped tail
# reaches e^130) leave no correct digit in the determinant on either side, and
# the GPU reports such a splat as non-finite geometry.  Capping changes about
# 0.1 % of the draws (per axis P(t3 > 9.9)); which pixels a capped splat
# covers changes, but the capped scene is rendered and differentiated exactly.
LOG_SCALE_CAP = math.log(50.0)


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config + 1000 * salt))


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------

def focal_for_fov(width: int, fov_x_deg: float = 60.0) -> float:
    return 0.5 * width / math.tan(math.radians(fov_x_deg) / 2.0)


def camera_from_pose(rot: np.ndarray, position: np.ndarray, width: int, height: int,
                     fov_x_deg: float = 60.0) -> dict:
    """World->camera matrix from camera axes (rows of ``rot``) and position."""
    rot = np.asarray(rot, dtype=np.float64)
    position = np.asarray(position, dtype=np.float64)
    vm = np.eye(4, dtype=np.float64)
    vm[:3, :3] = rot
    vm[:3, 3] = -rot @ position
    f = focal_for_fov(width, fov_x_deg)
    return dict(viewmat=vm.astype(np.float32), fx=np.float32(f), fy=np.float32(f),
                cx=np.float32(width / 2.0), cy=np.float32(height / 2.0),
                width=int(width), height=int(height))


def orbit_camera(radius: float, azimuth_deg: float, elevation_deg: float,
                 width: int, height: int, fov_x_deg: float = 60.0) -> dict:
    """Camera on a sphere around the origin, looking at the origin.

    World "up" is -y so that the identity rotation (camera at (0, 0, -r)) has
    image +y pointing down.  Azimuth 0 / elevation 0 is the point (0, 0, -r).
    """
    az = math.radians(azimuth_deg)
    el = math.radians(elevation_deg)
    pos = np.array([radius * math.cos(el) * math.sin(az),
                    -radius * math.sin(el),
                    -radius * math.cos(el) * math.cos(az)])
    fwd = -pos / np.linalg.norm(pos)
    down = np.array([0.0, 1.0, 0.0])
    y_c = down - down.dot(fwd) * fwd
    y_c /= np.linalg.norm(y_c)
    x_c = np.cross(y_c, fwd)
    rot = np.stack([x_c, y_c, fwd])
    return camera_from_pose(rot, pos, width, height, fov_x_deg)


def crop_camera(cam: dict, x0: int, y0: int, width: int, height: int) -> dict:
    """The sub-window [x0, x0+width) x [y0, y0+height) rendered as its own camera."""
    out = dict(cam)
    out["cx"] = np.float32(float(cam["cx"]) - x0)
    out["cy"] = np.float32(float(cam["cy"]) - y0)
    out["width"] = int(width)
    out["height"] = int(height)
    return out


# --------------------------------------------------------------------------
# building blocks (each documents its draw order)
# --------------------------------------------------------------------------

def _normal(rng, mu, sigma, shape):
    """Normal draws in float32 (numpy's float32 ziggurat)."""
    z = rng.standard_normal(shape, dtype=np.float32)
    if sigma != 1.0:
        z *= np.float32(sigma)
    if mu != 0.0:
        z += np.float32(mu)
    return z


def _student_t3(rng, shape):
    """Student-t with 3 degrees of freedom from its definition Z / sqrt(chi2_3 / 3)."""
    z = _normal(rng, 0.0, 1.0, shape)
    chi2 = np.sum(_normal(rng, 0.0, 1.0, (3,) + tuple(shape)) ** 2, axis=0)
    return z / np.sqrt(chi2 / 3.0)


def _unit_quats(rng, n):
    q = _normal(rng, 0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _uniform_ball(rng, n, radius):
    d = _normal(rng, 0.0, 1.0, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    return d * r[:, None]


def _clusters(rng, n_clusters, per_cluster, sigma, centre_radius, keep_radius):
    """Isotropic clusters; points outside ``keep_radius`` are redrawn around
    their own cluster centre until every point lies inside."""
    centres = _uniform_ball(rng, n_clusters, centre_radius)
    owner = np.repeat(np.arange(n_clusters), per_cluster)
    pts = centres[owner] + _normal(rng, 0.0, sigma, (owner.size, 3))
    bad = np.linalg.norm(pts, axis=1) > keep_radius
    while bad.any():
        idx = np.nonzero(bad)[0]
        pts[idx] = centres[owner[idx]] + _normal(rng, 0.0, sigma, (idx.size, 3))
        bad[idx] = np.linalg.norm(pts[idx], axis=1) > keep_radius
    return pts


def _shell(rng, n, r_lo, r_hi):
    d = _normal(rng, 0.0, 1.0, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * rng.uniform(r_lo, r_hi, n)[:, None]


def _sh_coeffs(rng, n, degree, rest_sigma):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3), np.float32)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh[:, 0, :] = (rgb - 0.5) / _Y00
    if k > 1:
        sh[:, 1:, :] = _normal(rng, 0.0, rest_sigma, (n, k - 1, 3))
    return sh


def _pack(means, log_scales, quats, opacity_logits, sh, mask_logits):
    n = means.shape[0]
    scores = np.zeros((n, 2))
    scores[:, 0] = mask_logits
    return dict(means=np.ascontiguousarray(means, np.float32),
                log_scales=np.ascontiguousarray(log_scales, np.float32),
                quats=np.ascontiguousarray(quats, np.float32),
                opacity_logits=np.ascontiguousarray(opacity_logits, np.float32),
                sh=np.ascontiguousarray(sh, np.float32),
                mask_scores=np.ascontiguousarray(scores, np.float32))


def _bernoulli_masks(rng, mask_logits):
    p = 1.0 / (1.0 + np.exp(-mask_logits))
    return (rng.uniform(0.0, 1.0, mask_logits.shape) < p).astype(np.float32)


def converged_mask_scores(n: int, pruned_fraction: float = 0.624, gap: float = 8.0, config: int = 4,
                          salt: int = 7) -> np.ndarray:
    """Mask scores [n, 2] as late training leaves them: the two scores of
    each Gaussian differ by `gap` (s0 - s1 = -gap for a seeded random
    `pruned_fraction` of the Gaussians, +gap for the rest).  The default
    fraction is the share of Gaussians the method removes on Mip-NeRF360
    (Sec. 4.2); which Gaussians they are is drawn uniformly, one uniform per
    Gaussian, since the synthetic scenes carry no learned contribution."""
    rng = rng_for(config, salt)
    u = rng.uniform(0.0, 1.0, n)
    scores = np.zeros((n, 2), np.float32)
    scores[:, 0] = np.where(u < pruned_fraction, -gap, gap)
    return scores


def _targets(rng, cams):
    return [rng.uniform(0.0, 1.0, (3, c["height"], c["width"])).astype(np.float32) for c in cams]


def _heavy_tail_log_scales(rng, n):
    t = _student_t3(rng, (n, 3))
    return np.minimum(-4.0 + 0.8 * t, LOG_SCALE_CAP)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def tiny_scene(n: int = 4096, width: int = 128, height: int = 128, config: int = 1) -> dict:
    """Tiny scene, one plain view (4096 Gaussians, 128x128, SH degree 0).

    Draw order: means U[-1,1]^3; log-scales N(-3, 0.3); quaternions
    normalize(N(0,1)^4); opacity logits N(0,1); base colour U[0,1]; mask
    logits N(1,1); Bernoulli mask uniforms; target image U[0,1].
    Camera at (0, 0, -4) looking along +z (identity rotation), 60 deg fov.
    """
    rng = rng_for(config)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = _normal(rng, -3.0, 0.3, (n, 3))
    quats = _unit_quats(rng, n)
    opac = _normal(rng, 0.0, 1.0, n)
    sh = _sh_coeffs(rng, n, 0, 0.0)
    mlog = _normal(rng, 1.0, 1.0, n)
    scene = _pack(means, log_scales, quats, opac, sh, mlog)
    scene["masks"] = _bernoulli_masks(rng, mlog)
    scene["sh_degree"] = 0
    cams = [orbit_camera(4.0, 0.0, 0.0, width, height)]
    scene["cameras"] = cams
    scene["targets"] = _targets(rng, cams)
    scene["name"] = f"tiny{n}_{width}x{height}_sh0"
    return scene


def object_scene(n: int = 200_000, width: int = 800, height: int = 800, config: int = 2) -> dict:
    """Object scene (200k Gaussians in 64 clusters, SH degree 3, one 800x800 view).

    Draw order: 64 cluster centres uniform in the unit ball; points
    centre + N(0, 0.15^2 I) redrawn until |p| <= 1; log-scales N(-4.5, 0.6);
    quaternions; opacity logits N(0, 1.5); base colour U[0,1] then the 15
    higher SH coefficients per channel N(0, 0.2); mask logits N(2, 1);
    Bernoulli mask uniforms; target U[0,1].  Orbit camera radius 4,
    azimuth 30 deg, elevation 20 deg.
    """
    rng = rng_for(config)
    per = n // 64
    assert per * 64 == n, "object scene needs a multiple of 64 Gaussians"
    means = _clusters(rng, 64, per, 0.15, 1.0, 1.0)
    log_scales = _normal(rng, -4.5, 0.6, (n, 3))
    quats = _unit_quats(rng, n)
    opac = _normal(rng, 0.0, 1.5, n)
    sh = _sh_coeffs(rng, n, 3, 0.2)
    mlog = _normal(rng, 2.0, 1.0, n)
    scene = _pack(means, log_scales, quats, opac, sh, mlog)
    scene["masks"] = _bernoulli_masks(rng, mlog)
    scene["sh_degree"] = 3
    cams = [orbit_camera(4.0, 30.0, 20.0, width, height)]
    scene["cameras"] = cams
    scene["targets"] = _targets(rng, cams)
    scene["name"] = f"object{n}_{width}x{height}_sh3"
    return scene


def _unbounded_gaussians(rng, n):
    n_fg = (n * 4) // 5
    n_fg -= n_fg % 64
    n_bg = n - n_fg
    fg = _clusters(rng, 64, n_fg // 64, 0.45, 3.0, 3.0)
    bg = _shell(rng, n_bg, 20.0, 50.0)
    means = np.concatenate([fg, bg])
    log_scales = _heavy_tail_log_scales(rng, n)
    quats = _unit_quats(rng, n)
    opac = _normal(rng, 0.0, 1.5, n)
    sh = _sh_coeffs(rng, n, 3, 0.2)
    return means, log_scales, quats, opac, sh


UNEVEN_VIEW_SIZES = [(640, 480), (800, 800), (1024, 768), (1264, 832),
                     (1296, 840), (1600, 1060), (960, 540), (512, 512)]


def unbounded_scene(n: int = 1_500_000, width: int = 1264, height: int = 832,
                    config: int = 3) -> dict:
    """Unbounded scene (1.5M Gaussians, heavy-tailed scales, SH degree 3).

    Draw order: 80% foreground = 64 cluster centres uniform in the radius-3
    ball, points centre + N(0, 0.45^2 I) redrawn until |p| <= 3; 20%
    background shell (uniform direction, radius U[20, 50]); log-scales
    -4 + 0.8 * t(df=3) per axis, capped at ln 50; quaternions; opacity logits
    N(0, 1.5); SH degree 3 as in the object scene; mask logits N(1.5, 1.2);
    target U[0,1].  Masks are not drawn here: they come from the
    straight-through Gumbel sampler with a (seed, step) counter.  Orbit camera
    radius 5, azimuth 0, elevation 15 deg.
    """
    rng = rng_for(config)
    means, log_scales, quats, opac, sh = _unbounded_gaussians(rng, n)
    mlog = _normal(rng, 1.5, 1.2, n)
    scene = _pack(means, log_scales, quats, opac, sh, mlog)
    scene["sh_degree"] = 3
    cams = [orbit_camera(5.0, 0.0, 15.0, width, height)]
    scene["cameras"] = cams
    scene["targets"] = _targets(rng, cams)
    scene["gumbel_tau"] = 0.5
    scene["name"] = f"unbounded{n}_{width}x{height}_sh3"
    return scene


def batched_scene(n: int = 1_000_000, sizes=None, config: int = 4) -> dict:
    """Eight uneven views of the 1M-Gaussian unbounded scene.

    Same draw order as ``unbounded_scene`` (with its own seed); views at
    azimuth k*45 deg, elevation 15 deg, radius 5, sizes 640x480, 800x800,
    1024x768, 1264x832, 1296x840, 1600x1060, 960x540, 512x512; one target per
    view drawn after the mask logits.
    """
    sizes = UNEVEN_VIEW_SIZES if sizes is None else sizes
    rng = rng_for(config)
    means, log_scales, quats, opac, sh = _unbounded_gaussians(rng, n)
    mlog = _normal(rng, 1.5, 1.2, n)
    scene = _pack(means, log_scales, quats, opac, sh, mlog)
    scene["sh_degree"] = 3
    cams = [orbit_camera(5.0, 45.0 * k, 15.0, w, h) for k, (w, h) in enumerate(sizes)]
    scene["cameras"] = cams
    scene["targets"] = _targets(rng, cams)
    scene["gumbel_tau"] = 0.5
    scene["name"] = f"batched{n}_{len(cams)}views_sh3"
    return scene


def training_scene(n: int = 3_000_000, width: int = 1920, height: int = 1080,
                   n_poses: int = 32, config: int = 5) -> dict:
    """Training workload: a ground-truth set and a perturbed trainee.

    Ground truth: the unbounded recipe with seed ``SEED_BASE + 5`` (all masks
    1).  Trainee (seed ``SEED_BASE + 5 + 1000``), draw order: mean noise
    N(0, 0.02^2), log-scale noise N(0, 0.1^2), DC noise N(0, 0.1^2), fresh
    opacity logits N(0, 1), mask logits N(1.5, 1.2), then 32 poses with
    azimuth U[0, 360) and elevation U[5, 30] deg on the radius-5 orbit.
    """
    rng = rng_for(config)
    gt_means, gt_ls, gt_q, gt_op, gt_sh = _unbounded_gaussians(rng, n)
    gt = _pack(gt_means, gt_ls, gt_q, gt_op, gt_sh, np.full(n, 30.0))
    gt["masks"] = np.ones(n, np.float32)
    rng2 = rng_for(config, salt=1)
    means = gt_means + _normal(rng2, 0.0, 0.02, (n, 3))
    ls = np.minimum(gt_ls + _normal(rng2, 0.0, 0.1, (n, 3)), LOG_SCALE_CAP)
    sh = gt_sh.copy()
    sh[:, 0, :] += _normal(rng2, 0.0, 0.1, (n, 3))
    opac = _normal(rng2, 0.0, 1.0, n)
    mlog = _normal(rng2, 1.5, 1.2, n)
    trainee = _pack(means, ls, gt_q, opac, sh, mlog)
    az = rng2.uniform(0.0, 360.0, n_poses)
    el = rng2.uniform(5.0, 30.0, n_poses)
    cams = [orbit_camera(5.0, a, e, width, height) for a, e in zip(az, el)]
    return dict(gt=gt, trainee=trainee, cameras=cams, sh_degree=3, gumbel_tau=0.5,
                name=f"train{n}_{width}x{height}")


def small_scene(n: int, width: int, height: int, seed: int, sh_degree: int = 1,
                log_scale_mean: float = -2.0, depth: float = 4.0,
                opacity_mean: float = 0.0, n_views: int = 1) -> dict:
    """Small scene for unit tests: n Gaussians in [-1,1]^3, any SH degree."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = _normal(rng, log_scale_mean, 0.3, (n, 3))
    quats = _unit_quats(rng, n)
    opac = _normal(rng, opacity_mean, 1.0, n)
    sh = _sh_coeffs(rng, n, sh_degree, 0.3)
    mlog = _normal(rng, 1.0, 1.0, n)
    scene = _pack(means, log_scales, quats, opac, sh, mlog)
    scene["masks"] = _bernoulli_masks(rng, mlog)
    scene["sh_degree"] = sh_degree
    cams = [orbit_camera(depth, 360.0 * k / max(n_views, 1), 10.0 * k, width, height)
            for k in range(n_views)]
    scene["cameras"] = cams
    scene["targets"] = _targets(rng, cams)
    scene["name"] = f"small{n}_{width}x{height}_sh{sh_degree}_s{seed}"
    return scene


CONFIGS = {1: tiny_scene, 2: object_scene, 3: unbounded_scene, 4: batched_scene}
