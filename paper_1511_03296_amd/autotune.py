"""Autotuner of the batched PCG's block shape.

A batch plan sizes each lane width's PCG launch (K consecutive channels of a
vertex per lane) at one block per `tiles` tiles of its images' estimated
vertices; the launch's blocks are then shared among the images on the
device, in proportion to their true work.  Fewer tiles per block gives more,
shorter blocks; more gives fewer, longer-running ones that amortise each
block's prologue.  The best value depends on the batch's sizes and channel
counts, so it is measured on the caller's own batch: a coordinate search over
the lane widths present, timing one pass of the batch for each candidate with
the other widths at their current choice.
"""
from __future__ import annotations

import time

import torch

from . import _lib as L

CANDIDATES = (4, 8, 16, 32)


def lane_widths(channels) -> list[int]:
    """Lane widths of the given channel counts, widest first."""
    return sorted({int(L.lib.bs_lane_width(int(c))) for c in channels}, reverse=True)


def set_tiles(K: int, tiles: int) -> None:
    """Tiles per block for lane width K (0: the library default)."""
    L.check(L.lib.bs_batch_set_tiles_per_block(int(K), int(tiles)),
            "bs_batch_set_tiles_per_block")


def current() -> dict:
    return {K: int(L.lib.bs_batch_tiles_per_block(K)) for K in (1, 2, 3, 4)}


def reset() -> None:
    for K in (1, 2, 3, 4):
        set_tiles(K, 0)


def _time(step, repeats: int) -> float:
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_batch(step, channels, candidates=CANDIDATES, repeats: int = 2) -> dict:
    """Chooses the tiles per block of every lane width in `channels` by
    timing `step()` (one pass over the batch through the batch engine).
    Returns {K: {"tiles": chosen, "seconds": {candidate: best time}}}; the
    choices stay in effect for later batch calls."""
    out = {}
    for K in lane_widths(channels):
        times = {}
        for t in candidates:
            set_tiles(K, t)
            step()   # warm-up with this shape
            times[t] = _time(step, repeats)
        pick = min(times, key=times.get)
        set_tiles(K, pick)
        out[K] = {"tiles": pick, "seconds": {t: round(v, 5) for t, v in times.items()}}
    return out


def tune_plan(trial, channels, candidates=CANDIDATES, repeats: int = 2) -> dict:
    """As tune_batch, for batch plans, which read the tiles per block when
    they are made: `trial()` makes the plan anew and returns a function that
    runs one pass of it."""
    out = {}
    for K in lane_widths(channels):
        times = {}
        for t in candidates:
            set_tiles(K, t)
            step = trial()
            step()
            times[t] = _time(step, repeats)
        pick = min(times, key=times.get)
        set_tiles(K, pick)
        out[K] = {"tiles": pick, "seconds": {t: round(v, 5) for t, v in times.items()}}
    return out
