"""FP64 CPU oracle for masked rasterization (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The product path (``paper_2412_20522_amd``) never
imports it.  The C source ``maskgs_oracle.c`` holds all arithmetic; this module
only marshals numpy arrays through ctypes.

Functions mirror the stages of the method (see the C file's header for the
paper passage each follows).  All returned floating arrays are float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maskgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Camera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 16), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class Settings(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("sh_degree", C.c_int32), ("exact_mode", C.c_int32),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float), ("q_max", C.c_float),
                ("near_plane", C.c_float), ("dilation", C.c_float), ("jac_clamp", C.c_float),
                ("lambda_floor", C.c_float), ("bg", C.c_float * 3), ("margin", C.c_float), ("margin_t", C.c_float)]


@dataclass
class RasterSettings:
    """Rasterization constants.  Defaults: 16x16 tiles, alpha filter 1/255,
    alpha clamp 0.99, early stop at T < 1e-4, Q cut 9 (3 sigma), near plane
    0.2, EWA dilation 0.3, Jacobian clamp 1.3 x tan(fov/2), eigenvalue floor
    0.1, black background."""
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 0
    exact_mode: bool = False
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    q_max: float = 9.0
    near_plane: float = 0.2
    dilation: float = 0.3
    jac_clamp: float = 1.3
    lambda_floor: float = 0.1
    bg: tuple = (0.0, 0.0, 0.0)
    margin: float = 1e-5
    margin_t: float = 2e-4

    def c(self) -> Settings:
        s = Settings()
        s.tile_w, s.tile_h, s.sh_degree, s.exact_mode = self.tile_w, self.tile_h, self.sh_degree, int(self.exact_mode)
        s.alpha_min, s.alpha_max, s.t_min, s.q_max = self.alpha_min, self.alpha_max, self.t_min, self.q_max
        s.near_plane, s.dilation, s.jac_clamp, s.lambda_floor = (self.near_plane, self.dilation, self.jac_clamp,
                                                                 self.lambda_floor)
        for i in range(3):
            s.bg[i] = self.bg[i]
        s.margin = self.margin
        s.margin_t = self.margin_t
        return s


def camera_c(cam: dict) -> Camera:
    c = Camera()
    vm = np.asarray(cam["viewmat"], np.float32).reshape(16)
    for i in range(16):
        c.viewmat[i] = float(vm[i])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _lib.orc_build_lists.restype = C.c_int64
        _lib.orc_total_tiles.restype = C.c_int64
        _lib.orc_l1_loss.restype = C.c_double
        _lib.orc_psnr.restype = C.c_double
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------

def sh_basis(degree: int, dirs):
    dirs = _f64(dirs).reshape(-1, 3)
    k = (degree + 1) ** 2
    vals = np.zeros((dirs.shape[0], k))
    grads = np.zeros((dirs.shape[0], k, 3))
    lib().orc_sh_basis(C.c_int(degree), C.c_int64(dirs.shape[0]), _p(dirs), _p(vals), _p(grads))
    return vals, grads


@dataclass
class Projected:
    mean2d: np.ndarray
    depth_bits: np.ndarray
    conic: np.ndarray
    cov2d: np.ndarray
    radius: np.ndarray
    opacity: np.ndarray
    color: np.ndarray
    color_clamped: np.ndarray
    valid: np.ndarray

    @property
    def depth(self):
        return self.depth_bits.view(np.float32)


def project(scene: dict, cam: dict, st: RasterSettings) -> Projected:
    n = scene["means"].shape[0]
    out = Projected(np.zeros((n, 2)), np.zeros(n, np.uint32), np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n),
                    np.zeros(n), np.zeros((n, 3)), np.zeros((n, 3), np.uint8), np.zeros(n, np.uint8))
    args = [_f64(scene[k]) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    camc, stc = camera_c(cam), st.c()
    lib().orc_project_fwd(C.c_int64(n), *[_p(a) for a in args], C.byref(camc), C.byref(stc), _p(out.mean2d),
                          _p(out.depth_bits), _p(out.conic), _p(out.cov2d), _p(out.radius), _p(out.opacity),
                          _p(out.color), _p(out.color_clamped), _p(out.valid))
    return out


@dataclass
class Lists:
    tiles_touched: np.ndarray  # [V*n] int64
    keys: np.ndarray           # [K] uint64
    vals: np.ndarray           # [K] uint32 (record = view*n + g)
    ranges: np.ndarray         # [total_tiles, 2] uint32
    total_tiles: int


def total_tiles(widths, heights, st: RasterSettings) -> int:
    w = np.ascontiguousarray(widths, np.int32)
    h = np.ascontiguousarray(heights, np.int32)
    stc = st.c()
    return int(lib().orc_total_tiles(C.c_int(len(w)), _p(w), _p(h), C.byref(stc)))


def build_lists(widths, heights, n: int, mean2d, radius, depth_bits, valid, st: RasterSettings) -> Lists:
    """Tile lists for V views; per-record inputs have leading size V*n."""
    w = np.ascontiguousarray(widths, np.int32)
    h = np.ascontiguousarray(heights, np.int32)
    V = len(w)
    mean2d, radius = _f64(mean2d).reshape(V * n, 2), _f64(radius).reshape(V * n)
    depth_bits = np.ascontiguousarray(depth_bits, np.uint32).reshape(V * n)
    valid = np.ascontiguousarray(valid, np.uint8).reshape(V * n)
    stc = st.c()
    tt = np.zeros(V * n, np.int64)
    L = lib()
    K = L.orc_build_lists(C.c_int(V), C.c_int64(n), _p(w), _p(h), _p(mean2d), _p(radius), _p(depth_bits),
                          _p(valid), C.byref(stc), _p(tt), None, None, C.c_int64(0), None)
    T = total_tiles(w, h, st)
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    ranges = np.zeros((T, 2), np.uint32)
    K2 = L.orc_build_lists(C.c_int(V), C.c_int64(n), _p(w), _p(h), _p(mean2d), _p(radius), _p(depth_bits),
                           _p(valid), C.byref(stc), _p(tt), _p(keys), _p(vals), C.c_int64(K), _p(ranges))
    assert K2 == K
    return Lists(tt, keys[:K], vals[:K], ranges, T)


@dataclass
class FwdOut:
    image: np.ndarray      # packed per view [3, H, W]
    t_final: np.ndarray    # packed per view [H, W]
    last: np.ndarray
    examined: np.ndarray
    n_blend: np.ndarray
    flags: np.ndarray


def _splat_args(mean2d, conic, opacity, color, mask):
    return [_f64(mean2d), _f64(conic), _f64(opacity), _f64(color), _f64(mask)]


def render_fwd(widths, heights, n: int, mean2d, conic, opacity, color, mask, lists: Lists,
               st: RasterSettings) -> FwdOut:
    w = np.ascontiguousarray(widths, np.int32)
    h = np.ascontiguousarray(heights, np.int32)
    P = int(np.sum(w.astype(np.int64) * h))
    out = FwdOut(np.zeros(3 * P), np.zeros(P), np.zeros(P, np.int64), np.zeros(P, np.int64), np.zeros(P, np.int64),
                 np.zeros(P, np.uint8))
    stc = st.c()
    vals = np.ascontiguousarray(lists.vals, np.uint32)
    ranges = np.ascontiguousarray(lists.ranges, np.uint32)
    lib().orc_render_fwd(C.c_int(len(w)), _p(w), _p(h), C.byref(stc), C.c_int64(n),
                         *[_p(a) for a in _splat_args(mean2d, conic, opacity, color, mask)], _p(vals), _p(ranges),
                         _p(out.image), _p(out.t_final), _p(out.last), _p(out.examined), _p(out.n_blend),
                         _p(out.flags))
    return out


def importance(widths, heights, n: int, mean2d, conic, opacity, color, mask, lists: Lists, st: RasterSettings):
    """Per Gaussian, the sum and the maximum over every pixel of every view of
    the blending weight M_i alpha_i T_i (the alpha T of score-based pruning,
    Sec. 2; Sec. 3.4).  Returns (imp_sum [n], imp_max [n])."""
    w = np.ascontiguousarray(widths, np.int32)
    h = np.ascontiguousarray(heights, np.int32)
    s, m = np.zeros(n), np.zeros(n)
    stc = st.c()
    vals = np.ascontiguousarray(lists.vals, np.uint32)
    ranges = np.ascontiguousarray(lists.ranges, np.uint32)
    lib().orc_importance(C.c_int(len(w)), _p(w), _p(h), C.byref(stc), C.c_int64(n),
                         *[_p(a) for a in _splat_args(mean2d, conic, opacity, color, mask)], _p(vals), _p(ranges),
                         _p(s), _p(m))
    return s, m


def scene_importance(scene: dict, cams: list, mask, st: RasterSettings):
    """importance() of a scene: projection and lists as in run_pipeline."""
    n = scene["means"].shape[0]
    projs = [project(scene, c, st) for c in cams]
    widths = [c["width"] for c in cams]
    heights = [c["height"] for c in cams]
    m2d, con, opa, col, rad, dbits, val = stack_projected(projs)
    lists = build_lists(widths, heights, n, m2d, rad, dbits, val, st)
    return importance(widths, heights, n, m2d, con, opa, col, _f64(mask).reshape(-1), lists, st)


@dataclass
class BwdOut:
    d_mean2d: np.ndarray
    d_conic: np.ndarray
    d_opacity: np.ndarray
    d_color: np.ndarray
    d_mask: np.ndarray
    touched_flagged: np.ndarray


def render_bwd(widths, heights, n: int, mean2d, conic, opacity, color, mask, lists: Lists, dl_dimage,
               st: RasterSettings) -> BwdOut:
    w = np.ascontiguousarray(widths, np.int32)
    h = np.ascontiguousarray(heights, np.int32)
    V = len(w)
    R = V * n
    out = BwdOut(np.zeros((R, 2)), np.zeros((R, 3)), np.zeros(R), np.zeros((R, 3)), np.zeros(n),
                 np.zeros(R, np.uint8))
    stc = st.c()
    vals = np.ascontiguousarray(lists.vals, np.uint32)
    ranges = np.ascontiguousarray(lists.ranges, np.uint32)
    lib().orc_render_bwd(C.c_int(V), _p(w), _p(h), C.byref(stc), C.c_int64(n),
                         *[_p(a) for a in _splat_args(mean2d, conic, opacity, color, mask)], _p(vals), _p(ranges),
                         _p(_f64(dl_dimage)), _p(out.d_mean2d), _p(out.d_conic), _p(out.d_opacity),
                         _p(out.d_color), _p(out.d_mask), _p(out.touched_flagged))
    return out


def render_pixels_direct(proj: Projected, mask, pixels, st: RasterSettings):
    """Colour, final transmittance and blend count at the given (x, y) pixels of one view."""
    px = np.ascontiguousarray(pixels, np.int32).reshape(-1, 2)
    m = px.shape[0]
    rgb, tf, nb = np.zeros((m, 3)), np.zeros(m), np.zeros(m, np.int64)
    stc = st.c()
    n = proj.mean2d.shape[0]
    lib().orc_render_pixels_direct(C.c_int64(n), _p(_f64(proj.mean2d)), _p(_f64(proj.conic)),
                                   _p(_f64(proj.opacity)), _p(_f64(proj.color)),
                                   _p(np.ascontiguousarray(proj.depth_bits, np.uint32)),
                                   _p(np.ascontiguousarray(proj.valid, np.uint8)), _p(_f64(mask)), C.byref(stc),
                                   C.c_int64(m), _p(px), _p(rgb), _p(tf), _p(nb))
    return rgb, tf, nb


@dataclass
class ParamGrads:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray


def project_bwd(scene: dict, cams: list, st: RasterSettings, d_mean2d, d_conic, d_opacity, d_color) -> ParamGrads:
    n = scene["means"].shape[0]
    V = len(cams)
    k = (st.sh_degree + 1) ** 2
    g = ParamGrads(np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n), np.zeros((n, k, 3)))
    args = [_f64(scene[key]) for key in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    cam_arr = (Camera * V)(*[camera_c(c) for c in cams])
    stc = st.c()
    lib().orc_project_bwd(C.c_int(V), C.c_int64(n), *[_p(a) for a in args], cam_arr, C.byref(stc),
                          _p(_f64(d_mean2d)), _p(_f64(d_conic)), _p(_f64(d_opacity)), _p(_f64(d_color)),
                          _p(g.means), _p(g.log_scales), _p(g.quats), _p(g.opacity_logits), _p(g.sh))
    return g


def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, np.uint32).reshape(4)
    k = np.ascontiguousarray(key, np.uint32).reshape(2)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sample_masks(scores, tau: float, seed: int, step: int, return_noise: bool = False):
    s = _f64(scores).reshape(-1, 2)
    n = s.shape[0]
    m, y, g = np.zeros(n), np.zeros(n), np.zeros((n, 2))
    lib().orc_sample_masks(C.c_int64(n), _p(s), C.c_double(tau), C.c_uint64(seed), C.c_uint64(step), _p(m), _p(y),
                           _p(g))
    return (m, y, g) if return_noise else (m, y)


def threshold_masks(scores, threshold: float):
    """Straight-through alternative of the ablation (Sec. 4.3, Table 6):
    y = sigmoid(s0 - s1) and the deterministic mask [y > threshold]; with
    mask_grad at tau = 1 the gradient passes through the threshold as if it
    were the identity."""
    s = _f64(scores).reshape(-1, 2)
    n = s.shape[0]
    m, y = np.zeros(n), np.zeros(n)
    lib().orc_threshold_masks(C.c_int64(n), _p(s), C.c_double(threshold), _p(m), _p(y))
    return m, y


def prune_keep(scores, seed: int, step0: int, n_draws: int = 10):
    """Probabilistic pruning (Sec. 3.5, training and pruning): every Gaussian
    draws n_draws hard masks -- the draws of sample_masks at steps step0 ..
    step0 + n_draws - 1 -- and survives iff at least one of them is 1."""
    n = _f64(scores).reshape(-1, 2).shape[0]
    keep = np.zeros(n, bool)
    for d in range(n_draws):
        m, _ = sample_masks(scores, 1.0, seed, step0 + d)
        keep |= m > 0.5
    return keep


def mask_grad(d_mask, m_hard, y_soft, tau: float, lambda_m: float):
    n = len(m_hard)
    d = np.zeros((n, 2))
    lm = C.c_double(0.0)
    lib().orc_mask_grad(C.c_int64(n), _p(_f64(d_mask)), _p(_f64(m_hard)), _p(_f64(y_soft)), C.c_double(tau),
                        C.c_double(lambda_m), _p(d), C.byref(lm))
    return d, lm.value


def l1_loss(image, target):
    im = _f64(image).reshape(-1)
    tg = _f32(target).reshape(-1)
    d = np.zeros_like(im)
    loss = lib().orc_l1_loss(C.c_int64(im.size), _p(im), _p(tg), _p(d))
    return loss, d


def psnr(a, b) -> float:
    a, b = _f64(a).reshape(-1), _f64(b).reshape(-1)
    return float(lib().orc_psnr(C.c_int64(a.size), _p(a), _p(b)))


def adam(params, grads, m1, m2, lr, b1, b2, eps, step):
    """In-place Adam on float64 arrays."""
    for a in (params, grads, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(C.c_int64(params.size), _p(params), _p(grads), _p(m1), _p(m2), C.c_double(lr), C.c_double(b1),
                   C.c_double(b2), C.c_double(eps), C.c_int64(step))


# ---------------------------------------------------------------------------
# whole pipeline for one scene and a list of cameras
# ---------------------------------------------------------------------------

@dataclass
class Pipeline:
    proj: list = field(default_factory=list)   # Projected per view
    lists: Lists = None
    fwd: FwdOut = None
    bwd: BwdOut = None
    grads: ParamGrads = None
    loss: float = 0.0
    d_image: np.ndarray = None


def stack_projected(projs):
    return (np.concatenate([p.mean2d for p in projs]), np.concatenate([p.conic for p in projs]),
            np.concatenate([p.opacity for p in projs]), np.concatenate([p.color for p in projs]),
            np.concatenate([p.radius for p in projs]), np.concatenate([p.depth_bits for p in projs]),
            np.concatenate([p.valid for p in projs]))


def run_pipeline(scene: dict, cams: list, mask, st: RasterSettings, targets=None, dl_dimage=None,
                 backward: bool = True, mask_mode: str = "raster") -> Pipeline:
    """Projection, lists, forward, L1 loss (or a given image gradient),
    backward and projection backward, all in FP64.

    mask_mode "raster": masked rasterization (Eq. 3-4, gradient Eq. 6).
    mask_mode "opacity": the alternative of the ablation in Sec. 4.3 (Table
    7): the mask multiplies the opacity before rasterization, which then runs
    unmasked (mask 1); dL/dM follows by the chain rule through the product,
    dL/dM_i = sum over views of dL/d(M_i o_i) * o_i, and the opacity's own
    gradient takes the factor M_i."""
    if mask_mode not in ("raster", "opacity"):
        raise ValueError(mask_mode)
    n = scene["means"].shape[0]
    out = Pipeline()
    out.proj = [project(scene, c, st) for c in cams]
    widths = [c["width"] for c in cams]
    heights = [c["height"] for c in cams]
    m2d, con, opa, col, rad, dbits, val = stack_projected(out.proj)
    out.lists = build_lists(widths, heights, n, m2d, rad, dbits, val, st)
    mask = _f64(mask).reshape(-1)
    V = len(cams)
    if mask_mode == "opacity":
        opa_r, mask_r = opa * np.tile(mask, V), np.ones(n)
    else:
        opa_r, mask_r = opa, mask
    out.fwd = render_fwd(widths, heights, n, m2d, con, opa_r, col, mask_r, out.lists, st)
    if not backward:
        return out
    if dl_dimage is None:
        tgt = np.concatenate([np.asarray(t, np.float32).reshape(-1) for t in targets])
        out.loss, out.d_image = l1_loss(out.fwd.image, tgt)
    else:
        out.d_image = _f64(dl_dimage).reshape(-1)
    out.bwd = render_bwd(widths, heights, n, m2d, con, opa_r, col, mask_r, out.lists, out.d_image, st)
    d_opa = out.bwd.d_opacity
    if mask_mode == "opacity":
        out.bwd.d_mask = (d_opa * opa).reshape(V, n).sum(axis=0)
        d_opa = d_opa * np.tile(mask, V)
    out.grads = project_bwd(scene, cams, st, out.bwd.d_mean2d, out.bwd.d_conic, d_opa, out.bwd.d_color)
    return out
