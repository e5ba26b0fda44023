"""Rasterizer objects and the differentiable masked rasterization op.

``MaskedRasterize`` is the torch.autograd.Function of MaskGaussian's
training step (Sec. 3.3-3.5): it samples hard masks from two scores per
Gaussian with a straight-through Gumbel-Softmax, renders with masked
compositing (Eq. 3-4), and in backward returns gradients for every Gaussian
parameter and for the scores, through dL/dM (Eq. 6) and the mask-count loss
(Eq. 7-8).  Transmittance is recomputed in reverse inside the backward
kernel; nothing per pixel beyond the final transmittance and the last
blended entry is kept.
"""
from __future__ import annotations

import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import maskgs as M

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def image_sizes(cams: Sequence[dict]):
    return [(int(c["height"]), int(c["width"])) for c in cams]


def total_pixels(cams: Sequence[dict]) -> int:
    return sum(h * w for h, w in image_sizes(cams))


def split_views(flat: torch.Tensor, cams: Sequence[dict]):
    """Packed [3 * P] images -> list of [3, H, W] views (views, no copy)."""
    out, off = [], 0
    for h, w in image_sizes(cams):
        out.append(flat[off:off + 3 * h * w].view(3, h, w))
        off += 3 * h * w
    return out


@dataclass
class Grads:
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    masks: torch.Tensor


class Rasterizer:
    """A library context plus a pool of frames on one device."""

    def __init__(self, device: int = 0, **settings):
        self.device = device
        self.ctx = M.mgs_create(device)
        self.settings = M.settings_struct(**settings)
        self._free_frames = []

    def __del__(self):
        try:
            for f in self._free_frames:
                M.mgs_frame_destroy(f)
            M.mgs_destroy(self.ctx)
        except Exception:
            pass

    def set(self, **settings) -> None:
        for k, v in settings.items():
            if k == "bg":
                for i in range(3):
                    self.settings.bg[i] = float(v[i])
            else:
                setattr(self.settings, k, type(getattr(self.settings, k))(v))

    def acquire_frame(self):
        return self._free_frames.pop() if self._free_frames else M.mgs_frame_create(self.ctx)

    def release_frame(self, frame) -> None:
        self._free_frames.append(frame)

    # -- plain calls -------------------------------------------------------
    def forward(self, frame, params: dict, masks: torch.Tensor, cams: Sequence[dict],
                images: Optional[torch.Tensor] = None, t_final: Optional[torch.Tensor] = None) -> torch.Tensor:
        dev = params["means"].device
        if images is None:
            images = torch.empty(3 * total_pixels(cams), dtype=torch.float32, device=dev)
        g = M.gaussians_struct(*(params[k] for k in PARAM_KEYS), masks)
        M.mgs_forward(self.ctx, frame, g, cams, self.settings, images, t_final)
        return images

    def forward_importance(self, frame, params: dict, masks: torch.Tensor, cams: Sequence[dict],
                           images: Optional[torch.Tensor] = None, imp_sum: Optional[torch.Tensor] = None,
                           imp_max: Optional[torch.Tensor] = None):
        """forward() that also returns each Gaussian's sum and maximum of its
        blending weights M alpha T over every pixel of every view (the scores
        of score-based pruning): (images, imp_sum, imp_max)."""
        dev = params["means"].device
        n = params["means"].shape[0]
        if images is None:
            images = torch.empty(3 * total_pixels(cams), dtype=torch.float32, device=dev)
        if imp_sum is None:
            imp_sum = torch.empty(n, dtype=torch.float32, device=dev)
        if imp_max is None:
            imp_max = torch.empty(n, dtype=torch.float32, device=dev)
        g = M.gaussians_struct(*(params[k] for k in PARAM_KEYS), masks)
        M.mgs_forward_importance(self.ctx, frame, g, cams, self.settings, images, imp_sum, imp_max)
        return images, imp_sum, imp_max

    def backward(self, frame, params: dict, dl_dimages: torch.Tensor, out: Optional[Grads] = None,
                 records: Optional[torch.Tensor] = None, accumulate: bool = False) -> Grads:
        """records (optional, [n_views N, 9] float32) receives the per-record 2D
        gradients before the chain rule (dL/d(u, v), the stored conic,
        opacity and colour); accumulate adds the parameter and mask
        gradients to what `out` holds."""
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs the output gradients")
            out = Grads(*(torch.empty_like(params[k]) for k in PARAM_KEYS),
                        torch.empty(params["means"].shape[0], dtype=torch.float32, device=params["means"].device))
        gr = M.gradients_struct(out.means, out.log_scales, out.quats, out.opacity_logits, out.sh, out.masks,
                                records, accumulate)
        M.mgs_backward(self.ctx, frame, dl_dimages.contiguous(), gr)
        return out

    # -- fixed workspace, capture, tuning ------------------------------------
    def reserve(self, frame, slack: float = 1.25) -> None:
        """Fix the frame's workspace after a plain forward, so that forward and
        backward on it neither allocate nor synchronise (capturable)."""
        M.mgs_frame_reserve(self.ctx, frame, slack)

    def check(self, frame) -> None:
        """Raise if the last forward on the frame overflowed its workspace or
        projected non-finite geometry (synchronises)."""
        M.mgs_frame_check(self.ctx, frame)

    def autotune(self, frame, params: dict, masks: torch.Tensor, cams: Sequence[dict], dl_dimages: torch.Tensor,
                 images: Optional[torch.Tensor] = None, out: Optional[Grads] = None, apply: bool = True):
        """Time the compositing configurations on this workload; returns
        (settings as a dict, ms) and, with apply, makes them current."""
        dev = params["means"].device
        if images is None:
            images = torch.empty(3 * total_pixels(cams), dtype=torch.float32, device=dev)
        if out is None:
            out = Grads(*(torch.empty_like(params[k]) for k in PARAM_KEYS),
                        torch.empty(params["means"].shape[0], dtype=torch.float32, device=dev))
        g = M.gaussians_struct(*(params[k] for k in PARAM_KEYS), masks)
        gr = M.gradients_struct(out.means, out.log_scales, out.quats, out.opacity_logits, out.sh, out.masks)
        best, ms = M.mgs_autotune(self.ctx, frame, g, cams, self.settings, images, dl_dimages.contiguous(), gr)
        if apply:
            self.settings = best
        keys = ("tile_w", "tile_h", "batch_depth", "fwd_ppt", "bwd_ppt", "wide_tiles")
        return {k: getattr(best, k) for k in keys}, ms

    def count_evals(self, frame) -> dict:
        """examined / blended / blended_masked / bwd_examined of the last forward."""
        return M.mgs_frame_count_evals(self.ctx, frame)

    def stats(self, frame) -> dict:
        return M.mgs_frame_get_stats(frame)

    def sample_masks(self, scores: torch.Tensor, tau: float, seed: int, step: int,
                     step_offset: Optional[torch.Tensor] = None):
        """Hard and soft straight-through Gumbel masks; step_offset (int64
        device scalar, optional) is added to step on the device."""
        n = scores.shape[0]
        m = torch.empty(n, dtype=torch.float32, device=scores.device)
        y = torch.empty_like(m)
        M.mgs_sample_masks(self.ctx, scores.contiguous(), tau, seed, step, m, y, step_offset=step_offset)
        return m, y


class MaskedRasterize(torch.autograd.Function):
    """images, mask_loss = MaskedRasterize.apply(means, log_scales, quats,
    opacity_logits, sh, mask_scores, rasterizer, cams, tau, seed, step,
    frame=None, step_offset=None)

    images is the packed [3 * P] rendering of all views; mask_loss is the
    0-dim (mean M)^2 of Eq. (7), computed by the library, so a caller forms
    L = L_render + lambda_m * mask_loss (Eq. 8).  The hard masks are
    available as ``rasterizer.last_masks``.

    frame: a frame the caller owns (for a captured step, one with a fixed
    workspace, see Rasterizer.reserve); without one a frame is taken from the
    rasterizer's pool and given back after the backward, or when the graph
    is dropped without a backward (evaluation, no_grad).  step_offset: int64
    device scalar added to step when the masks are drawn.  Nothing in
    forward or backward reads a device value on the host, so a whole step
    (with the loss, backward and optimiser) can be captured into a hipGraph.
    """

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, mask_scores, rasterizer: Rasterizer,
                cams, tau: float, seed: int, step: int, frame=None, step_offset: Optional[torch.Tensor] = None):
        params = {"means": means.detach().contiguous(), "log_scales": log_scales.detach().contiguous(),
                  "quats": quats.detach().contiguous(), "opacity_logits": opacity_logits.detach().contiguous(),
                  "sh": sh.detach().contiguous()}
        m_hard, y_soft = rasterizer.sample_masks(mask_scores.detach(), tau, seed, step, step_offset)
        own = frame is None
        fr = rasterizer.acquire_frame() if own else frame
        try:
            images = rasterizer.forward(fr, params, m_hard, cams)
        except Exception:
            if own:
                rasterizer.release_frame(fr)
            raise
        mask_loss = torch.empty((), dtype=torch.float32, device=m_hard.device)
        M.mgs_mask_loss(rasterizer.ctx, m_hard, mask_loss)
        ctx.rasterizer = rasterizer
        ctx.frame = fr
        ctx.params = params
        ctx.tau = tau
        # a pooled frame goes back to the pool once: after the backward, or
        # when this node is freed without one
        ctx.release = weakref.finalize(ctx, rasterizer.release_frame, fr) if own else None
        ctx.save_for_backward(m_hard, y_soft)
        rasterizer.last_masks = m_hard
        return images, mask_loss

    @staticmethod
    def backward(ctx, dl_dimages, dl_dmask_loss):
        m_hard, y_soft = ctx.saved_tensors
        r: Rasterizer = ctx.rasterizer
        if dl_dimages is None:
            n_px = M.mgs_frame_get_stats(ctx.frame)["n_pixels"]
            dl_dimages = torch.zeros(3 * n_px, dtype=torch.float32, device=m_hard.device)
        g = r.backward(ctx.frame, ctx.params, dl_dimages.contiguous())
        if ctx.release is not None:
            ctx.release()
        ctx.frame = None
        d_scores = torch.empty(m_hard.shape[0], 2, dtype=torch.float32, device=m_hard.device)
        if dl_dmask_loss is None:
            M.mgs_mask_grad(r.ctx, g.masks, m_hard, y_soft, ctx.tau, 0.0, d_scores)
        else:
            # the weight of L_m stays on the device: lambda_m = 1 scaled by
            # the incoming gradient of mask_loss
            scale = dl_dmask_loss.detach().to(torch.float32).reshape(1).contiguous()
            M.mgs_mask_grad(r.ctx, g.masks, m_hard, y_soft, ctx.tau, 1.0, d_scores, lambda_scale=scale)
        return (g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, d_scores,
                None, None, None, None, None, None, None)


class L1Loss(torch.autograd.Function):
    """loss = L1Loss.apply(images, targets, rasterizer): the rendering loss
    mean |images - targets| (L_render of Eq. 8) and its gradient, both from
    the library's loss kernels (sign(0) = 0).  0-dim float32 result."""

    @staticmethod
    def forward(ctx, images, targets, rasterizer: Rasterizer):
        img = images.detach().contiguous()
        tgt = targets.detach().contiguous()
        loss = torch.empty((), dtype=torch.float32, device=img.device)
        M.mgs_l1_loss_grad(rasterizer.ctx, img, tgt, None, loss.reshape(1))
        ctx.rasterizer = rasterizer
        ctx.save_for_backward(img, tgt)
        return loss

    @staticmethod
    def backward(ctx, dl_dloss):
        img, tgt = ctx.saved_tensors
        d = torch.empty_like(img)
        M.mgs_l1_loss_grad(ctx.rasterizer.ctx, img, tgt, d, None,
                           grad_scale=dl_dloss.detach().to(torch.float32).reshape(1).contiguous())
        return d, None, None


def masked_rasterize(params: dict, mask_scores: torch.Tensor, rasterizer: Rasterizer, cams, tau: float = 0.5,
                     seed: int = 0, step: int = 0, frame=None, step_offset: Optional[torch.Tensor] = None):
    return MaskedRasterize.apply(params["means"], params["log_scales"], params["quats"], params["opacity_logits"],
                                 params["sh"], mask_scores, rasterizer, cams, tau, seed, step, frame, step_offset)
