"""Helpers shared by the GPU parity tests: run each stage of the HIP path
through the C ABI and feed the oracle the GPU's own upstream outputs
(widened exactly to FP64) for stage-wise comparison."""
from __future__ import annotations

import numpy as np
import torch

import oracle

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def M():
    from paper_2412_20522_amd import maskgs
    return maskgs


def settings_pair(**kw):
    """Matching oracle and library settings."""
    ost = oracle.RasterSettings(**{k: v for k, v in kw.items() if k in oracle.RasterSettings.__dataclass_fields__})
    lib_kw = {k: v for k, v in kw.items() if k not in ("margin", "margin_t")}
    gst = M().settings_struct(**lib_kw)
    return ost, gst


def to_device(scene: dict, masks=None) -> dict:
    d = {k: torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).cuda() for k in PARAM_KEYS}
    m = scene["masks"] if masks is None else masks
    d["masks"] = torch.from_numpy(np.ascontiguousarray(m, np.float32)).cuda()
    if "mask_scores" in scene:
        d["mask_scores"] = torch.from_numpy(np.ascontiguousarray(scene["mask_scores"], np.float32)).cuda()
    return d


def gstruct(dev: dict):
    return M().gaussians_struct(*(dev[k] for k in PARAM_KEYS), dev["masks"])


def gpu_project(ctx, dev, cams, gst):
    n = dev["means"].shape[0]
    R = n * len(cams)
    rec = torch.zeros(max(R, 1), 12, device="cuda")
    depth = torch.zeros(max(R, 1), device="cuda")
    radius = torch.zeros(max(R, 1), device="cuda")
    tiles = torch.zeros(max(R, 1), dtype=torch.int32, device="cuda")
    M().mgs_project(ctx, gstruct(dev), cams, gst, rec, depth, radius, tiles)
    torch.cuda.synchronize()
    return rec[:R], depth[:R], radius[:R], tiles[:R]


def total_tiles(cams, tw, th):
    return sum(((c["width"] + tw - 1) // tw) * ((c["height"] + th - 1) // th) for c in cams)


def gpu_lists(ctx, rec, depth, radius, tiles, n, cams, gst):
    """scan -> duplicate -> sort -> ranges, each through its stage entry point."""
    R = tiles.numel()
    offsets = torch.zeros(max(R, 1), dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    M().mgs_scan(ctx, tiles, offsets[:R], total)
    torch.cuda.synchronize()
    K = int(total.item())
    keys = torch.zeros(max(K, 1), dtype=torch.int64, device="cuda")
    vals = torch.zeros(max(K, 1), dtype=torch.int32, device="cuda")
    if K > 0:
        M().mgs_duplicate(ctx, rec, depth, radius, tiles, offsets[:R], n, cams, gst, keys[:K], vals[:K])
    T = total_tiles(cams, gst.tile_w, gst.tile_h)
    key_bits = 32 + max(1, int(np.ceil(np.log2(max(T, 2)))))
    if K > 1:
        M().mgs_sort(ctx, keys[:K], vals[:K], key_bits)
    ranges = torch.zeros(T, 2, dtype=torch.int32, device="cuda")
    M().mgs_tile_ranges(ctx, keys[:K], T, ranges)
    torch.cuda.synchronize()
    return offsets[:R], K, keys[:K], vals[:K], ranges


def conic_from_rec(r) -> np.ndarray:
    """Records keep the conic as (a, b / a, c - b^2 / a); back to (a, b, c)
    in FP64 (b exactly, c to FP64 rounding)."""
    r = np.asarray(r, np.float64)
    a, beta, gamma = r[:, 2], r[:, 3], r[:, 4]
    return np.stack([a, a * beta, gamma + (a * beta) * beta], 1)


def dstable_from_dabc(a, beta, d) -> np.ndarray:
    """Gradient w.r.t. the conic (A, B, C) -> gradient w.r.t. the stored
    (a, beta, gamma) = (A, B / A, C - B^2 / A), the basis the kernels
    accumulate in (chain rule through A = a, B = a beta, C = gamma + a beta^2)."""
    a, beta, d = np.asarray(a, np.float64), np.asarray(beta, np.float64), np.asarray(d, np.float64)
    dA, dB, dC = d[:, 0], d[:, 1], d[:, 2]
    return np.stack([dA + beta * dB + beta * beta * dC, a * dB + 2.0 * a * beta * dC, dC], 1)


def dabc_from_dstable(conic, d) -> np.ndarray:
    """Inverse of dstable_from_dabc at the conic (A, B, C)."""
    conic, d = np.asarray(conic, np.float64), np.asarray(d, np.float64)
    A, B = conic[:, 0], conic[:, 1]
    da, db, dg = d[:, 0], d[:, 1], d[:, 2]
    return np.stack([da - db * B / (A * A) + dg * (B / A) ** 2, db / A - 2.0 * dg * B / A, dg], 1)


def oracle_inputs_from_rec(rec: torch.Tensor):
    r = rec.detach().cpu().numpy().astype(np.float64)
    return dict(mean2d=r[:, 0:2].copy(), conic=conic_from_rec(r), opacity=r[:, 5].copy(), color=r[:, 8:11].copy(),
                mask=r[:, 6].copy())


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def assert_grad_close(g, o, exclude=None, rtol=2e-3, name=""):
    """Norm-wise relative error <= rtol over the whole tensor, and element-wise
    |g - o| <= rtol |o| + 1e-2 rtol rms(o) over the rows not excluded."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    assert g.shape == o.shape, (name, g.shape, o.shape)
    e = rel_err(g, o)
    assert e <= rtol, f"{name}: norm-wise relative error {e:.3e} > {rtol}"
    rms = np.sqrt(np.mean(o ** 2)) if o.size else 0.0
    keep = np.ones(o.shape[0], bool) if exclude is None else ~np.asarray(exclude, bool)
    gk, ok = g[keep], o[keep]
    bad = np.abs(gk - ok) > rtol * np.abs(ok) + 1e-2 * rtol * rms
    assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} elements off; worst "
                           f"{np.max(np.abs(gk - ok) - rtol * np.abs(ok)):.3e} (rms {rms:.3e})")
