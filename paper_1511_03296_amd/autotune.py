"""Autotuner of the batched PCG's launch shape.

Two choices are measured on the caller's own batch:
  - the lane width of each channel count (K consecutive channels of a vertex
    per lane, the channel stride padded to a multiple of K): wider lanes
    read the neighbour table once for more channels and issue wider loads,
    narrower ones avoid padding and hold fewer registers;
  - the tiles per block of each lane width's PCG launch: a batch plan sizes
    that launch at one block per `tiles` tiles of its images' estimated
    vertices, and the launch's blocks are then shared among the images on
    the device, in proportion to their true work.  Fewer tiles per block
    gives more, shorter blocks; more gives fewer, longer-running ones that
    amortise each block's prologue.
Each is a coordinate search: one choice at a time, timing passes of the batch
for every candidate with the others at their current setting.
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
    """Every lane width's tiles per block and every channel count's lane
    width back to the library defaults."""
    for K in (1, 2, 3, 4):
        set_tiles(K, 0)
    for C in range(1, 65):
        L.check(L.lib.bs_set_lane_width(C, 0), "bs_set_lane_width")


def lane_candidates(C: int) -> list[int]:
    """Lane widths worth trying for C channels: the default, every width
    that divides C (no padding) and 4 (float4 accesses)."""
    C = int(C)
    out = {lane_candidates_default(C)}
    for K in (1, 2, 3, 4):
        if K <= C and (C % K == 0 or K == 4):
            out.add(K)
    return sorted(out)


LANE_MARGIN = 0.02


def lane_candidates_default(C: int) -> int:
    """The library's default lane width of C channels (ignoring overrides)."""
    C = int(C)
    return C if C <= 2 else (4 if C % 4 == 0 else (3 if C % 3 == 0 else 4))


def set_lane(C: int, K: int) -> None:
    """Lane width K for C channels (0: the library's default rule)."""
    L.check(L.lib.bs_set_lane_width(int(C), int(K)), "bs_set_lane_width")


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


def tune_lanes(trial, channels, repeats: int = 2) -> dict:
    """Chooses the lane width of every channel count in `channels` (most
    channels first) by timing a pass of a batch plan made anew by `trial()`
    for each candidate.  Returns {C: {"lane": chosen, "seconds": {K: best
    time}}}; the choices stay in effect for later workspaces and plans."""
    out = {}
    for C in sorted({int(c) for c in channels}, reverse=True):
        cands = lane_candidates(C)
        if len(cands) < 2:
            continue
        times = {}
        for K in cands:
            set_lane(C, K)
            step = trial()
            step()
            times[K] = _time(step, repeats)
        # the default layout stays unless another is clearly faster (timing
        # noise between passes is about a per cent)
        default = lane_candidates_default(C)
        pick = min(times, key=times.get)
        if times[pick] > (1.0 - LANE_MARGIN) * times[default]:
            pick = default
        set_lane(C, pick)
        out[C] = {"lane": pick, "seconds": {K: round(v, 5) for K, v in times.items()}}
    return out


def tune_plan(trial, channels, candidates=CANDIDATES, repeats: int = 2,
              lanes: bool = False) -> dict:
    """As tune_batch, for batch plans, which read the tiles per block when
    they are made: `trial()` makes the plan anew and returns a function that
    runs one pass of it.  With `lanes`, tune_lanes runs first and its result
    is returned under the key "lanes"."""
    out = {}
    if lanes:
        out["lanes"] = tune_lanes(trial, channels, repeats)
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
