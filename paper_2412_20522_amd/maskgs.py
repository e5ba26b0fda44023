"""ctypes binding of libmaskgs.so (include/maskgs.h).

Argument marshalling only: every function below checks tensor placement,
dtype and contiguity, takes device pointers and the current HIP stream from
torch, and calls the C entry point of the same name.  All arithmetic runs in
the library's gfx950 kernels.  If the library is missing, importing this
module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaskgs.so")

MGS_MAX_VIEWS = 16

STATUS = {0: "MGS_OK", 1: "MGS_ERR_INVALID_ARG", 2: "MGS_ERR_OOM", 3: "MGS_ERR_CAPACITY", 4: "MGS_ERR_NONFINITE",
          5: "MGS_ERR_HIP", 6: "MGS_ERR_UNSUPPORTED", 7: "MGS_ERR_STATE"}


class MaskGSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class mgs_camera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 16), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class mgs_settings(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("batch_depth", C.c_int32), ("sh_degree", C.c_int32),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float), ("q_max", C.c_float),
                ("near_plane", C.c_float), ("dilation", C.c_float), ("jac_clamp", C.c_float),
                ("lambda_floor", C.c_float), ("bg", C.c_float * 3), ("exact_mode", C.c_int32),
                ("persistent", C.c_int32), ("fwd_ppt", C.c_int32), ("bwd_ppt", C.c_int32),
                ("wide_tiles", C.c_int32), ("stats", C.c_int32), ("tile_cull", C.c_int32),
                ("mask_mode", C.c_int32)]


class mgs_gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("masks", C.c_void_p), ("n", C.c_int64)]


class mgs_gradients(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_log_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacity_logits", C.c_void_p), ("d_sh", C.c_void_p), ("d_masks", C.c_void_p),
                ("d_records", C.c_void_p), ("accumulate", C.c_int32)]


class mgs_eval_counts(C.Structure):
    _fields_ = [("examined", C.c_int64), ("blended", C.c_int64), ("blended_masked", C.c_int64),
                ("bwd_examined", C.c_int64), ("evaluated", C.c_int64), ("bwd_evaluated", C.c_int64)]


STAGES = ("project", "depth_sort", "scan", "duplicate", "sort", "ranges", "composite_fwd", "composite_bwd",
          "project_bwd", "sample_masks", "mask_grad", "loss", "adam")
EXPORTS = {"records": 0, "depth": 1, "radius": 2, "tiles": 3, "values": 4, "ranges": 5, "t_final": 6, "last": 7,
           "stats": 8, "order": 9, "evals": 10}
REGION_TILES = 4  # side of the regions that list wide records, in tiles
MASK_RASTER = 0   # mgs_settings.mask_mode: masked rasterization (Eq. 3-4, 6)
MASK_OPACITY = 1  # mgs_settings.mask_mode: M multiplies the opacity (ablation, Sec. 4.3)
MGS_NUM_STAGES = len(STAGES)


class mgs_frame_stats(C.Structure):
    _fields_ = [("n_gaussians", C.c_int64), ("n_views", C.c_int64), ("n_records", C.c_int64),
                ("n_pixels", C.c_int64), ("n_instances", C.c_int64), ("total_tiles", C.c_int64),
                ("instance_capacity", C.c_int64), ("n_wide", C.c_int64), ("sort_passes", C.c_int32),
                ("tile_bits", C.c_int32)]


class mgs_adam_array(C.Structure):
    _fields_ = [("params", C.c_void_p), ("grads", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float)]


# name -> (restype, argtypes)
_VP, _I64, _U64, _I32, _F, _SZ = C.c_void_p, C.c_int64, C.c_uint64, C.c_int, C.c_float, C.c_size_t
_SIGS = {
    "mgs_version": (C.c_int, []),
    "mgs_default_settings": (C.c_int, [C.POINTER(mgs_settings)]),
    "mgs_create": (C.c_int, [C.c_int, C.POINTER(_VP)]),
    "mgs_destroy": (C.c_int, [_VP]),
    "mgs_last_error": (C.c_char_p, [_VP]),
    "mgs_frame_create": (C.c_int, [_VP, C.POINTER(_VP)]),
    "mgs_frame_destroy": (C.c_int, [_VP]),
    "mgs_frame_get_stats": (C.c_int, [_VP, C.POINTER(mgs_frame_stats)]),
    "mgs_forward": (C.c_int, [_VP, _VP, C.POINTER(mgs_gaussians), C.POINTER(mgs_camera), C.c_int,
                              C.POINTER(mgs_settings), _VP, _VP]),
    "mgs_forward_importance": (C.c_int, [_VP, _VP, C.POINTER(mgs_gaussians), C.POINTER(mgs_camera), C.c_int,
                                         C.POINTER(mgs_settings), _VP, _VP, _VP, _VP]),
    "mgs_backward": (C.c_int, [_VP, _VP, _VP, C.POINTER(mgs_gradients)]),
    "mgs_frame_reserve": (C.c_int, [_VP, _VP, C.c_double]),
    "mgs_frame_check": (C.c_int, [_VP, _VP]),
    "mgs_autotune": (C.c_int, [_VP, _VP, C.POINTER(mgs_gaussians), C.POINTER(mgs_camera), C.c_int,
                               C.POINTER(mgs_settings), _VP, _VP, C.POINTER(mgs_gradients),
                               C.POINTER(mgs_settings), C.POINTER(C.c_double)]),
    "mgs_frame_count_evals": (C.c_int, [_VP, _VP, C.POINTER(mgs_eval_counts)]),
    "mgs_frame_export": (C.c_int, [_VP, _VP, C.c_int, _VP, C.POINTER(_SZ)]),
    "mgs_profile_enable": (C.c_int, [_VP, C.c_int]),
    "mgs_profile_read": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "mgs_project": (C.c_int, [_VP, _VP, C.POINTER(mgs_gaussians), C.POINTER(mgs_camera), C.c_int,
                              C.POINTER(mgs_settings), _VP, _VP, _VP, _VP]),
    "mgs_scan_scratch_bytes": (_SZ, [_I64]),
    "mgs_scan": (C.c_int, [_VP, _VP, _VP, _I64, _VP, _VP, _VP]),
    "mgs_scan_noalloc": (C.c_int, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "mgs_duplicate": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _I64, C.POINTER(mgs_camera), C.c_int,
                                C.POINTER(mgs_settings), _VP, _VP, _I64]),
    "mgs_sort_scratch_bytes": (_SZ, [_I64]),
    "mgs_sort": (C.c_int, [_VP, _VP, _VP, _VP, _I64, C.c_int, _VP, _VP, _VP]),
    "mgs_tile_ranges": (C.c_int, [_VP, _VP, _VP, _I64, _I64, _VP]),
    "mgs_project_backward": (C.c_int, [_VP, _VP, C.POINTER(mgs_gaussians), C.POINTER(mgs_camera), C.c_int,
                                       C.POINTER(mgs_settings), _VP, C.POINTER(mgs_gradients)]),
    "mgs_sample_masks": (C.c_int, [_VP, _VP, _VP, _I64, _F, _U64, _U64, _VP, _VP, _VP]),
    "mgs_reduce_scratch_bytes": (_SZ, [_I64]),
    "mgs_prune_sample": (C.c_int, [_VP, _VP, _VP, _I64, _U64, _U64, C.c_int, _VP]),
    "mgs_threshold_masks": (C.c_int, [_VP, _VP, _VP, _I64, _F, _VP, _VP]),
    "mgs_compact_scratch_bytes": (_SZ, [_I64]),
    "mgs_compact_rows": (C.c_int, [_VP, _VP, _VP, _I64, C.c_int, _VP, _VP, _VP, _VP, _VP]),
    "mgs_mask_loss": (C.c_int, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "mgs_mask_grad": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _I64, _F, _F, _VP, _VP, _VP, _VP]),
    "mgs_l1_loss_grad": (C.c_int, [_VP, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "mgs_adam_step": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _I64, _F, _F, _F, _F, _I64]),
    "mgs_adam_step_multi": (C.c_int, [_VP, _VP, C.POINTER(mgs_adam_array), C.c_int, _F, _F, _F, _I64, _VP]),
    "mgs_step_advance": (C.c_int, [_VP, _VP, _VP, _I64]),
}

EXPORTED = tuple(_SIGS)


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first (python -m paper_2412_20522_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def lib() -> C.CDLL:
    return _lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t: Optional[torch.Tensor], dtype=torch.float32, name: str = "tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def camera_struct(cam: dict) -> mgs_camera:
    c = mgs_camera()
    vm = np.asarray(cam["viewmat"], np.float32).reshape(16)
    for i in range(16):
        c.viewmat[i] = float(vm[i])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


def cameras_array(cams: Sequence[dict]):
    if not 1 <= len(cams) <= MGS_MAX_VIEWS:
        raise ValueError(f"1..{MGS_MAX_VIEWS} views supported, got {len(cams)}")
    return (mgs_camera * len(cams))(*[camera_struct(c) for c in cams])


def settings_struct(**overrides) -> mgs_settings:
    s = mgs_settings()
    _check(None, _lib.mgs_default_settings(C.byref(s)))
    for k, v in overrides.items():
        if k == "bg":
            for i in range(3):
                s.bg[i] = float(v[i])
        elif not hasattr(s, k):
            raise KeyError(f"unknown setting {k}")
        else:
            setattr(s, k, type(getattr(s, k))(v))
    return s


def gaussians_struct(means, log_scales, quats, opacity_logits, sh, masks=None) -> mgs_gaussians:
    g = mgs_gaussians()
    n = means.shape[0]
    g.means = _ptr(means, name="means")
    g.log_scales = _ptr(log_scales, name="log_scales")
    g.quats = _ptr(quats, name="quats")
    g.opacity_logits = _ptr(opacity_logits, name="opacity_logits")
    g.sh = _ptr(sh, name="sh")
    g.masks = _ptr(masks, name="masks")
    g.n = n
    return g


def gradients_struct(d_means=None, d_log_scales=None, d_quats=None, d_opacity_logits=None, d_sh=None,
                     d_masks=None, d_records=None, accumulate: bool = False) -> mgs_gradients:
    gr = mgs_gradients()
    gr.accumulate = 1 if accumulate else 0
    gr.d_means = _ptr(d_means, name="d_means")
    gr.d_log_scales = _ptr(d_log_scales, name="d_log_scales")
    gr.d_quats = _ptr(d_quats, name="d_quats")
    gr.d_opacity_logits = _ptr(d_opacity_logits, name="d_opacity_logits")
    gr.d_sh = _ptr(d_sh, name="d_sh")
    gr.d_masks = _ptr(d_masks, name="d_masks")
    gr.d_records = _ptr(d_records, name="d_records")
    return gr


def _check(ctx, status: int):
    if status != 0:
        msg = _lib.mgs_last_error(ctx)
        raise MaskGSError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def mgs_version() -> int:
    return _lib.mgs_version()


def mgs_default_settings() -> mgs_settings:
    return settings_struct()


def mgs_create(device: int = 0):
    h = C.c_void_p()
    _check(None, _lib.mgs_create(device, C.byref(h)))
    return h


def mgs_destroy(ctx) -> None:
    _lib.mgs_destroy(ctx)


def mgs_last_error(ctx) -> str:
    m = _lib.mgs_last_error(ctx)
    return m.decode() if m else ""


def mgs_frame_create(ctx):
    h = C.c_void_p()
    _check(ctx, _lib.mgs_frame_create(ctx, C.byref(h)))
    return h


def mgs_frame_destroy(frame) -> None:
    _lib.mgs_frame_destroy(frame)


def mgs_frame_get_stats(frame) -> dict:
    s = mgs_frame_stats()
    _check(None, _lib.mgs_frame_get_stats(frame, C.byref(s)))
    return {k: getattr(s, k) for k, _ in mgs_frame_stats._fields_}


def mgs_forward(ctx, frame, g: mgs_gaussians, cams: Sequence[dict], st: mgs_settings, images: torch.Tensor,
                t_final: Optional[torch.Tensor] = None, stream=None) -> None:
    ca = cameras_array(cams)
    _check(ctx, _lib.mgs_forward(frame, _stream(stream), C.byref(g), ca, len(cams), C.byref(st),
                                 _ptr(images, name="images"), _ptr(t_final, name="t_final")))


def mgs_forward_importance(ctx, frame, g: mgs_gaussians, cams: Sequence[dict], st: mgs_settings,
                           images: torch.Tensor, imp_sum: torch.Tensor, imp_max: torch.Tensor,
                           t_final: Optional[torch.Tensor] = None, stream=None) -> None:
    """mgs_forward plus per-Gaussian sum and maximum of the blending weights
    M alpha T over every pixel of every view (imp_sum, imp_max: [n] float32)."""
    ca = cameras_array(cams)
    _check(ctx, _lib.mgs_forward_importance(frame, _stream(stream), C.byref(g), ca, len(cams), C.byref(st),
                                            _ptr(images, name="images"), _ptr(t_final, name="t_final"),
                                            _ptr(imp_sum, name="imp_sum"), _ptr(imp_max, name="imp_max")))


def mgs_backward(ctx, frame, dl_dimages: torch.Tensor, grads: mgs_gradients, stream=None) -> None:
    _check(ctx, _lib.mgs_backward(frame, _stream(stream), _ptr(dl_dimages, name="dl_dimages"), C.byref(grads)))


def mgs_frame_reserve(ctx, frame, slack: float = 1.25, stream=None) -> None:
    _check(ctx, _lib.mgs_frame_reserve(frame, _stream(stream), C.c_double(slack)))


def mgs_frame_check(ctx, frame, stream=None) -> None:
    _check(ctx, _lib.mgs_frame_check(frame, _stream(stream)))


def mgs_autotune(ctx, frame, g: mgs_gaussians, cams: Sequence[dict], base: mgs_settings, images: torch.Tensor,
                 dl_dimages: torch.Tensor, grads: mgs_gradients, stream=None):
    """Returns (best settings, its forward + backward time in ms)."""
    ca = cameras_array(cams)
    best = mgs_settings()
    ms = C.c_double()
    _check(ctx, _lib.mgs_autotune(frame, _stream(stream), C.byref(g), ca, len(cams), C.byref(base),
                                  _ptr(images, name="images"), _ptr(dl_dimages, name="dl_dimages"), C.byref(grads),
                                  C.byref(best), C.byref(ms)))
    return best, ms.value


def mgs_frame_count_evals(ctx, frame, stream=None) -> dict:
    out = mgs_eval_counts()
    _check(ctx, _lib.mgs_frame_count_evals(frame, _stream(stream), C.byref(out)))
    return {k: int(getattr(out, k)) for k, _ in mgs_eval_counts._fields_}


_EXPORT_DTYPES = {"records": torch.float32, "depth": torch.float32, "radius": torch.float32, "tiles": torch.int32,
                  "values": torch.int32, "ranges": torch.int32, "t_final": torch.float32, "last": torch.int32,
                  "stats": torch.int32, "order": torch.int32,
                  "evals": torch.int32}


def mgs_frame_export(ctx, frame, what: str, stream=None) -> torch.Tensor:
    """A copy of one array of the frame's last forward (u32 arrays as int32)."""
    code = EXPORTS[what]
    nbytes = C.c_size_t()
    _check(ctx, _lib.mgs_frame_export(frame, _stream(stream), code, None, C.byref(nbytes)))
    dt = _EXPORT_DTYPES[what]
    esize = torch.tensor([], dtype=dt).element_size()
    out = torch.empty(max(nbytes.value // esize, 1), dtype=dt, device="cuda")
    _check(ctx, _lib.mgs_frame_export(frame, _stream(stream), code, C.c_void_p(out.data_ptr()), C.byref(nbytes)))
    return out[:nbytes.value // esize]


def mgs_profile_enable(ctx, on: bool = True) -> None:
    _check(ctx, _lib.mgs_profile_enable(ctx, 1 if on else 0))


def mgs_profile_read(ctx) -> dict:
    """{stage name: (total ms, launches)} since the last enable/read."""
    ms = (C.c_double * MGS_NUM_STAGES)()
    n = (C.c_int64 * MGS_NUM_STAGES)()
    _check(ctx, _lib.mgs_profile_read(ctx, ms, n))
    return {STAGES[i]: (float(ms[i]), int(n[i])) for i in range(MGS_NUM_STAGES)}


def mgs_project(ctx, g: mgs_gaussians, cams, st, rec, depth, radius, tiles, stream=None) -> None:
    ca = cameras_array(cams)
    _check(ctx, _lib.mgs_project(ctx, _stream(stream), C.byref(g), ca, len(cams), C.byref(st), _ptr(rec, name="rec"),
                                 _ptr(depth, name="depth"), _ptr(radius, name="radius"),
                                 _ptr(tiles, torch.int32, "tiles")))


def mgs_scan(ctx, inp: torch.Tensor, out: torch.Tensor, total: torch.Tensor, stream=None) -> None:
    n = inp.numel()
    scratch = torch.empty(int(_lib.mgs_scan_scratch_bytes(n)), dtype=torch.uint8, device=inp.device)
    _check(ctx, _lib.mgs_scan(ctx, _stream(stream), _ptr(inp, torch.int32, "in"), n, _ptr(out, torch.int32, "out"),
                              _ptr(total, torch.int64, "total"), _ptr(scratch, torch.uint8, "scratch")))


SCAN_NOALLOC_MAX_N = 33419264  # MGS_SCAN_NOALLOC_MAX_N


def mgs_scan_noalloc(ctx, inp: torch.Tensor, out: torch.Tensor, total: Optional[torch.Tensor] = None,
                     stream=None) -> None:
    """mgs_scan with the library's fixed per-GPU scratch (allocates nothing)."""
    _check(ctx, _lib.mgs_scan_noalloc(ctx, _stream(stream), _ptr(inp, torch.int32, "in"), inp.numel(),
                                      _ptr(out, torch.int32, "out"), _ptr(total, torch.int64, "total")))


def mgs_duplicate(ctx, rec, depth, radius, tiles, offsets, n: int, cams, st, keys, vals, stream=None) -> None:
    ca = cameras_array(cams)
    _check(ctx, _lib.mgs_duplicate(ctx, _stream(stream), _ptr(rec, name="rec"), _ptr(depth, name="depth"),
                                   _ptr(radius, name="radius"), _ptr(tiles, torch.int32, "tiles"),
                                   _ptr(offsets, torch.int32, "offsets"), n, ca, len(cams), C.byref(st),
                                   _ptr(keys, torch.int64, "keys"), _ptr(vals, torch.int32, "vals"), keys.numel()))


def mgs_sort(ctx, keys, vals, key_bits: int, stream=None) -> None:
    K = keys.numel()
    scratch = torch.empty(int(_lib.mgs_sort_scratch_bytes(K)), dtype=torch.uint8, device=keys.device)
    ka = torch.empty_like(keys)
    va = torch.empty_like(vals)
    _check(ctx, _lib.mgs_sort(ctx, _stream(stream), _ptr(keys, torch.int64, "keys"), _ptr(vals, torch.int32, "vals"),
                              K, key_bits, _ptr(ka, torch.int64, "keys_alt"), _ptr(va, torch.int32, "vals_alt"),
                              _ptr(scratch, torch.uint8, "scratch")))


def mgs_tile_ranges(ctx, keys, total_tiles: int, ranges, stream=None) -> None:
    _check(ctx, _lib.mgs_tile_ranges(ctx, _stream(stream), _ptr(keys, torch.int64, "keys"), keys.numel(),
                                     total_tiles, _ptr(ranges, torch.int32, "ranges")))


def mgs_project_backward(ctx, g: mgs_gaussians, cams, st, d_rec, grads: mgs_gradients, stream=None) -> None:
    ca = cameras_array(cams)
    _check(ctx, _lib.mgs_project_backward(ctx, _stream(stream), C.byref(g), ca, len(cams), C.byref(st),
                                          _ptr(d_rec, name="d_rec"), C.byref(grads)))


def mgs_sample_masks(ctx, scores, tau: float, seed: int, step: int, m_hard, y_soft, step_offset=None,
                     stream=None) -> None:
    """step_offset (optional): int64 device scalar added to step on the device."""
    _check(ctx, _lib.mgs_sample_masks(ctx, _stream(stream), _ptr(scores, name="scores"), scores.shape[0], tau,
                                      seed, step, _ptr(step_offset, torch.int64, "step_offset"),
                                      _ptr(m_hard, name="m_hard"), _ptr(y_soft, name="y_soft")))


def mgs_threshold_masks(ctx, scores, threshold: float, m_hard, y_soft, stream=None) -> None:
    """Deterministic straight-through masks: m_hard = [sigmoid(s0 - s1) > threshold]."""
    _check(ctx, _lib.mgs_threshold_masks(ctx, _stream(stream), _ptr(scores, name="scores"), scores.shape[0],
                                         threshold, _ptr(m_hard, name="m_hard"), _ptr(y_soft, name="y_soft")))


def mgs_prune_sample(ctx, scores, seed: int, step0: int, n_draws: int, keep, stream=None) -> None:
    """keep [n] int32 (0/1): Gaussians with at least one of n_draws hard masks."""
    _check(ctx, _lib.mgs_prune_sample(ctx, _stream(stream), _ptr(scores, name="scores"), scores.shape[0], seed,
                                      step0, n_draws, _ptr(keep, torch.int32, "keep")))


def mgs_compact_rows(ctx, keep, ins, outs, n_kept=None, scratch=None, stream=None) -> None:
    """Stable compaction of the rows of every tensor in `ins` (leading size n,
    float32, contiguous) with keep != 0 into the matching tensor of `outs`;
    n_kept (int64 device scalar, optional) receives the number kept."""
    n = keep.numel()
    if len(ins) != len(outs):
        raise ValueError("ins and outs differ in length")
    widths = []
    for a, b in zip(ins, outs):
        if a.shape[0] != n:
            raise ValueError("every array needs one row per Gaussian")
        widths.append(max(a.numel() // max(n, 1), 1))
        if b.numel() < a.numel():
            raise ValueError("an output array is smaller than its input")
    if scratch is None:
        scratch = torch.empty(int(_lib.mgs_compact_scratch_bytes(n)), dtype=torch.uint8, device=keep.device)
    k = len(ins)
    pin = (C.c_void_p * max(k, 1))(*[_ptr(a, name="in") for a in ins])
    pout = (C.c_void_p * max(k, 1))(*[_ptr(b, name="out") for b in outs])
    pw = (C.c_int * max(k, 1))(*widths)
    _check(ctx, _lib.mgs_compact_rows(ctx, _stream(stream), _ptr(keep, torch.int32, "keep"), n, k, pin, pout, pw,
                                      _ptr(n_kept, torch.int64, "n_kept"), _ptr(scratch, torch.uint8, "scratch")))


def mgs_mask_loss(ctx, m_hard, loss_m, scratch=None, stream=None) -> None:
    n = m_hard.numel()
    if scratch is None:
        scratch = torch.empty(int(_lib.mgs_reduce_scratch_bytes(n)), dtype=torch.uint8, device=m_hard.device)
    _check(ctx, _lib.mgs_mask_loss(ctx, _stream(stream), _ptr(m_hard, name="m_hard"), n, _ptr(loss_m, name="loss_m"),
                                   _ptr(scratch, torch.uint8, "scratch")))


def mgs_mask_grad(ctx, d_masks, m_hard, y_soft, tau: float, lambda_m: float, d_scores, loss_m=None,
                  scratch=None, lambda_scale=None, stream=None) -> None:
    """lambda_scale (optional): float32 device scalar multiplying lambda_m."""
    n = m_hard.numel()
    if scratch is None:
        scratch = torch.empty(int(_lib.mgs_reduce_scratch_bytes(n)), dtype=torch.uint8, device=m_hard.device)
    _check(ctx, _lib.mgs_mask_grad(ctx, _stream(stream), _ptr(d_masks, name="d_masks"), _ptr(m_hard, name="m_hard"),
                                   _ptr(y_soft, name="y_soft"), n, tau, lambda_m,
                                   _ptr(lambda_scale, name="lambda_scale"), _ptr(d_scores, name="d_scores"),
                                   _ptr(loss_m, name="loss_m"), _ptr(scratch, torch.uint8, "scratch")))


def mgs_l1_loss_grad(ctx, images, targets, d_images, loss=None, scratch=None, grad_scale=None, stream=None) -> None:
    """d_images may be None (loss only); grad_scale (optional): float32 device
    scalar multiplying the gradient."""
    m = images.numel()
    if targets.numel() != m or (d_images is not None and d_images.numel() != m):
        raise ValueError("images, targets and d_images differ in size")
    if scratch is None:
        scratch = torch.empty(int(_lib.mgs_reduce_scratch_bytes(m)), dtype=torch.uint8, device=images.device)
    _check(ctx, _lib.mgs_l1_loss_grad(ctx, _stream(stream), _ptr(images, name="images"),
                                      _ptr(targets, name="targets"), m, _ptr(d_images, name="d_images"),
                                      _ptr(grad_scale, name="grad_scale"), _ptr(loss, name="loss"),
                                      _ptr(scratch, torch.uint8, "scratch")))


def mgs_adam_step_multi(ctx, groups, beta1: float, beta2: float, eps: float, step: int, step_offset=None,
                        stream=None) -> None:
    """groups: sequence of (params, grads, m, v, lr) with float32 device
    tensors of equal size per group; step_offset (optional): int64 device
    scalar added to step for the bias corrections."""
    arr = (mgs_adam_array * max(len(groups), 1))()
    for i, (p, g, m1, m2, lr) in enumerate(groups):
        if not (p.numel() == g.numel() == m1.numel() == m2.numel()):
            raise ValueError(f"group {i}: params, grads and moments differ in size")
        arr[i].params = _ptr(p, name="params")
        arr[i].grads = _ptr(g, name="grads")
        arr[i].m = _ptr(m1, name="m")
        arr[i].v = _ptr(m2, name="v")
        arr[i].n = p.numel()
        arr[i].lr = float(lr)
    _check(ctx, _lib.mgs_adam_step_multi(ctx, _stream(stream), arr, len(groups), beta1, beta2, eps, step,
                                         _ptr(step_offset, torch.int64, "step_offset")))


def mgs_step_advance(ctx, counter, delta: int = 1, stream=None) -> None:
    _check(ctx, _lib.mgs_step_advance(ctx, _stream(stream), _ptr(counter, torch.int64, "counter"), delta))


def mgs_adam_step(ctx, params, grads, m, v, lr: float, beta1: float, beta2: float, eps: float, step: int,
                  stream=None) -> None:
    _check(ctx, _lib.mgs_adam_step(ctx, _stream(stream), _ptr(params, name="params"), _ptr(grads, name="grads"),
                                   _ptr(m, name="m"), _ptr(v, name="v"), params.numel(), lr, beta1, beta2, eps,
                                   step))
