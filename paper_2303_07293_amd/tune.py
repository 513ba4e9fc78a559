"""Velocity-block shape tuner for prepared searches.

The stacking kernels are compiled for several velocity-block shapes (see
`sst_shapes`); which one is fastest depends on the problem: the grid is
padded to whole blocks, and a block's frame window is widened by the spread
of its shifts (a block too spread to stage in LDS falls back to reads
through L2).  `tune_plan` prepares a plan with every shape, times a run of
each on the caller's frames and keeps the fastest; the choice is cached per
geometry, so later calls for the same geometry prepare the chosen shape
only.  Every shape gives the same candidate lists bit for bit.
"""

from __future__ import annotations

import hashlib
from typing import Dict, Optional, Tuple

import numpy as np

from .binding import SstPlan, sst_plan_detect, sst_shapes

_choice: Dict[str, int] = {}
_timings: Dict[str, Tuple[float, ...]] = {}


def _key(n: int, h: int, w: int, t, t_ref: float, vx, vy, k_max: int) -> str:
    hsh = hashlib.sha256()
    hsh.update(np.asarray([n, h, w, k_max], dtype=np.int64).tobytes())
    for a in (t, [t_ref], vx, vy):
        hsh.update(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).tobytes())
    return hsh.hexdigest()


def tune_plan(frames, t, t_ref: float, vx, vy, threshold: float, min_coverage: int = 0, k_max: int = 64,
              reps: int = 2, scale=None) -> SstPlan:
    """A prepared plan (SstPlan) for the geometry of `frames` ([n][h][w] on
    the GPU) with the fastest velocity-block shape.  The first call for a
    geometry times `reps` runs of every shape (after one warm-up run) on the
    current stream; an unstaged shape is timed only if no shape is staged."""
    import torch
    n, h, w = frames.shape
    key = _key(n, h, w, t, t_ref, vx, vy, k_max)
    dev = frames.device
    if key in _choice:
        return sst_plan_detect(n, h, w, t, t_ref, vx, vy, threshold, min_coverage, k_max, device=dev,
                               shape=_choice[key])
    plans = [sst_plan_detect(n, h, w, t, t_ref, vx, vy, threshold, min_coverage, k_max, device=dev, shape=sh)
             for sh in range(len(sst_shapes()))]
    any_staged = any(p.staged for p in plans)
    best: Optional[SstPlan] = None
    best_ms = float("inf")
    times = []
    for p in plans:
        if any_staged and not p.staged:
            times.append(float("inf"))
            continue
        p.run(frames, scale=scale)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            p.run(frames, scale=scale)
        e1.record()
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / reps
        times.append(ms)
        if ms < best_ms:
            best, best_ms = p, ms
    for p in plans:
        if p is not best:
            p.close()
    _choice[key] = best.shape
    _timings[key] = tuple(times)
    return best


def tuned_shape(n: int, h: int, w: int, t, t_ref: float, vx, vy, k_max: int = 64) -> Optional[int]:
    """The shape chosen for this geometry so far (None if not tuned yet)."""
    return _choice.get(_key(n, h, w, t, t_ref, vx, vy, k_max))


def tuning_times(n: int, h: int, w: int, t, t_ref: float, vx, vy, k_max: int = 64) -> Optional[Tuple[float, ...]]:
    """Milliseconds per run of each shape measured when the geometry was
    tuned (inf: not timed), or None."""
    return _timings.get(_key(n, h, w, t, t_ref, vx, vy, k_max))
