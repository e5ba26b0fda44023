"""Probabilistic pruning and the mask-loss schedules (Sec. 3.5; Sec. 4.1,
implementation details) on top of the C ABI.

Pruning draws n (10) hard masks per Gaussian with the mask sampler and
removes the Gaussians that were never sampled; the survivors' rows of every
per-Gaussian array (parameters, mask scores, optimiser state) are compacted
in order on the device (`mgs_prune_sample`, `mgs_compact_rows`).  The
schedules are host logic: which mask-loss weight an iteration uses, and
which iterations prune.
"""
from __future__ import annotations

from typing import Dict, Tuple

import torch

from . import maskgs as M

# Mask-loss weight schedules of the experiments: (weight, first iteration,
# last iteration exclusive); None = every iteration.
LAMBDA_SCHEDULES = {
    "alpha": (0.1, 19_000, 20_000),
    "beta": (0.0005, None, None),
    "gamma": (0.001, None, None),
}


def lambda_m(iteration: int, variant: str) -> float:
    """lambda_m at `iteration` for the schedule `variant` ("alpha", "beta",
    "gamma"); 0 outside the schedule's range."""
    w, lo, hi = LAMBDA_SCHEDULES[variant]
    if lo is None:
        return w
    return w if lo <= iteration < hi else 0.0


def prune_due(iteration: int, densify_from: int = 500, densify_until: int = 15_000, densify_every: int = 100,
              after_every: int = 1000) -> bool:
    """Whether `iteration` prunes: at every densification step (every
    `densify_every` iterations in [densify_from, densify_until]) and every
    `after_every` iterations after densification has ended."""
    if iteration <= 0:
        return False
    if densify_from <= iteration <= densify_until:
        return iteration % densify_every == 0
    return iteration > densify_until and iteration % after_every == 0


def prune(ctx, scores: torch.Tensor, arrays: Dict[str, torch.Tensor], seed: int, step0: int, n_draws: int = 10,
          stream=None) -> Tuple[Dict[str, torch.Tensor], torch.Tensor, int]:
    """Draws the keep mask from `scores` [N, 2] and compacts `scores` and every
    array of `arrays` (leading size N) to the survivors, in order.  Returns the
    compacted arrays (with "scores"), the keep mask [N] (int32) and the number
    kept (one synchronisation)."""
    n = scores.shape[0]
    keep = torch.empty(n, dtype=torch.int32, device=scores.device)
    M.mgs_prune_sample(ctx, scores, seed, step0, n_draws, keep, stream=stream)
    names = ["scores", *arrays.keys()]
    ins = [scores, *arrays.values()]
    outs = [torch.empty_like(t) for t in ins]
    n_kept = torch.zeros(1, dtype=torch.int64, device=scores.device)
    M.mgs_compact_rows(ctx, keep, ins, outs, n_kept=n_kept, stream=stream)
    k = int(n_kept.item())
    return {name: t[:k] for name, t in zip(names, outs)}, keep, k
