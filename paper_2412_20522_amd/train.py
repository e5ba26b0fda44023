"""Differentiable training steps of MaskGaussian on the device.

One step (Sec. 3.3-3.5) draws straight-through Gumbel masks from two scores
per Gaussian, renders a batch of views with masked rasterization (Eq. 3-4),
forms L = L_render + lambda_m L_m (Eq. 7-8, L_render the L1 loss), runs the
backward through Eq. (6) and updates every attribute and both mask scores
with Adam.  Everything runs in the library's kernels; torch provides the
tensors, the autograd graph that ties the two Functions together and the
stream capture.

The masks' counter step and Adam's bias-correction step come from one int64
counter on the device, advanced at the end of every step, so a step captured
once into a hipGraph per camera batch replays as a fresh step each time.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import torch

from . import maskgs as M
from .raster import PARAM_KEYS, L1Loss, MaskedRasterize, Rasterizer, total_pixels

TRAIN_KEYS = PARAM_KEYS + ("mask_scores",)

# Learning rates.  The paper trains with the optimiser settings of its 3DGS
# code base (Sec. 4.1) and gives no mask learning rate; these follow that
# lineage's defaults (positions scaled by the scene extent, one rate for all
# SH coefficients) and take 1e-2 for the mask scores.
DEFAULT_LRS = {"means": 1.6e-4 * 5.0, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3,
               "mask_scores": 1e-2}
ADAM_BETAS = (0.9, 0.999)
ADAM_EPS = 1e-15


@dataclass
class StepRecord:
    """Device scalars of one step (read on the host only when asked)."""
    l1: torch.Tensor
    mask_loss: torch.Tensor


@dataclass
class Trainer:
    """Training state of one scene: parameters (leaf tensors), Adam moments,
    the device step counter and a frame of its own.

    params: float32 device tensors keyed by TRAIN_KEYS (updated in place).
    batches: camera lists, one per step in rotation; targets: the packed
    [3 * P] target images of each batch.
    """
    rast: Rasterizer
    params: Dict[str, torch.Tensor]
    batches: List[Sequence[dict]]
    targets: List[torch.Tensor]
    tau: float = 0.5
    seed: int = 0
    lambda_m: float = 0.1
    lrs: Dict[str, float] = field(default_factory=lambda: dict(DEFAULT_LRS))

    def __post_init__(self):
        if len(self.batches) != len(self.targets):
            raise ValueError("one target per camera batch")
        for b, (cams, t) in enumerate(zip(self.batches, self.targets)):
            if t.numel() != 3 * total_pixels(cams):
                raise ValueError(f"batch {b}: target of {t.numel()} values for {3 * total_pixels(cams)}")
        dev = self.params["means"].device
        for k in TRAIN_KEYS:
            p = self.params[k]
            if p.dtype != torch.float32 or not p.is_contiguous() or p.device != dev:
                raise ValueError(f"{k} must be a contiguous float32 tensor on {dev}")
            p.requires_grad_(True)
        self.m1 = {k: torch.zeros_like(self.params[k]) for k in TRAIN_KEYS}
        self.m2 = {k: torch.zeros_like(self.params[k]) for k in TRAIN_KEYS}
        # steps taken so far; masks use seed and this counter, Adam step it + 1
        self.counter = torch.zeros(1, dtype=torch.int64, device=dev)
        self.frame = self.rast.acquire_frame()
        self.graphs: Dict[int, tuple] = {}
        self.steps_done = 0

    # -- one step ---------------------------------------------------------
    def _body(self, b: int) -> StepRecord:
        p = self.params
        for k in TRAIN_KEYS:
            p[k].grad = None
        images, mask_loss = MaskedRasterize.apply(p["means"], p["log_scales"], p["quats"], p["opacity_logits"],
                                                  p["sh"], p["mask_scores"], self.rast, self.batches[b], self.tau,
                                                  self.seed, 0, self.frame, self.counter)
        self.last_images = images.detach()
        l1 = L1Loss.apply(images, self.targets[b], self.rast)
        loss = l1 + self.lambda_m * mask_loss
        loss.backward()
        groups = [(p[k].detach(), p[k].grad, self.m1[k], self.m2[k], self.lrs[k]) for k in TRAIN_KEYS]
        M.mgs_adam_step_multi(self.rast.ctx, groups, ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS, 1,
                              step_offset=self.counter)
        M.mgs_step_advance(self.rast.ctx, self.counter, 1)
        return StepRecord(l1.detach(), mask_loss.detach())

    def step(self, b: Optional[int] = None) -> StepRecord:
        """One step on batch b (default: the next in rotation), replaying its
        captured graph when there is one.  A replay returns the graph's own
        scalars (and leaves its images in last_images), which the next replay
        of the same graph overwrites."""
        if b is None:
            b = self.steps_done % len(self.batches)
        self.steps_done += 1
        if b in self.graphs:
            g, rec, images = self.graphs[b]
            g.replay()
            self.last_images = images
            return rec
        return self._body(b)

    # -- fixed workspace and capture ----------------------------------------
    def reserve(self, slack: float = 1.5) -> None:
        """Fix the frame's workspace for every batch: forwards (no parameter
        change) of each batch find the one with most list entries, whose
        counts times `slack` size the reservation."""
        p = {k: self.params[k].detach() for k in PARAM_KEYS}
        best, best_k = 0, -1
        self.rast.reserve(self.frame, 0.0)  # back to the growing workspace
        for b, cams in enumerate(self.batches):
            m, _ = self.rast.sample_masks(self.params["mask_scores"].detach(), self.tau, self.seed, 0, self.counter)
            self.rast.forward(self.frame, p, m, cams)
            k = self.rast.stats(self.frame)["n_instances"]
            if k > best_k:
                best, best_k = b, k
        m, _ = self.rast.sample_masks(self.params["mask_scores"].detach(), self.tau, self.seed, 0, self.counter)
        self.rast.forward(self.frame, p, m, self.batches[best])
        self.rast.reserve(self.frame, slack)

    def capture(self, batches: Optional[Sequence[int]] = None) -> None:
        """Capture one whole step (masks, forward, losses, backward, Adam,
        counter) per camera batch into a hipGraph.  Needs reserve() first;
        capturing runs nothing."""
        batches = range(len(self.batches)) if batches is None else batches
        for b in batches:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                rec = self._body(b)
            self.graphs[b] = (g, rec, self.last_images)

    def check(self) -> None:
        """Raise if a forward outgrew the fixed workspace (synchronises)."""
        self.rast.check(self.frame)

    def warmup(self, steps: int) -> None:
        """Eager steps on a side stream (they are real training steps), as
        capture requires before the first graph."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(steps):
                self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def close(self) -> None:
        self.graphs.clear()
        self.rast.reserve(self.frame, 0.0)
        self.rast.release_frame(self.frame)
