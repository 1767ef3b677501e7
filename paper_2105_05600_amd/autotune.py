"""Launch-shape autotuner for the fitness kernel.

The fitness kernel is compiled for a few shapes (particles per wavefront x
points per lane per step).  For a workload (volume, point set, particle
count) the tuner times every compiled shape on the GPU with HIP events,
keeps the fastest, sets it process-wide (rose_fitness_set_shape) and caches
the choice in a JSON file keyed by device, volume size/format, lookup,
point count and particle count, so later runs skip the timing.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import torch

from paper_2105_05600_amd import rose

SHAPES = [(4, 2), (8, 2), (4, 4), (4, 8), (2, 4), (8, 4), (64, 4), (64, 8), (64, 16)]  # (64, U): one particle per lane
# the batched tracker's candidates: the fixed shapes of its persistent launch,
# and the switching mode (0, 0), in which each sequence with enough work per
# iteration takes the single path's launches of its own and the rest share
# the persistent launch at the switching mode's points-across shape
BATCH_SHAPES = [(4, 2), (8, 2), (4, 4), (4, 8), (8, 4), (64, 8), (0, 0)]
# the tracker's candidates: the points-across shapes and the switching mode
# (0, 0).  The fixed particle-per-lane shapes are left out: they win only on
# iterations with a small search footprint and lose on wide ones, and one
# timed frame does not show a sequence's mix of the two (on the room
# workload a frame of small axis lengths timed 64x8 at 0.24 ms against 0.32
# for the switching mode, while over 60 frames 64x8 averaged 0.79 ms per
# step against 0.62); the switching mode uses that kernel exactly where it wins.
TRACK_SHAPES = [s for s in SHAPES if s[0] != 64] + [(0, 0)]
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _key(vol, m: int, n: int, lookup: int) -> str:
    dev = torch.cuda.get_device_properties(0)
    arch = getattr(dev, "gcnArchName", dev.name).split(":")[0]
    nx, ny, nz = vol.dims
    # bucket the point count so nearby frames share an entry
    mb = 1 << max(0, int(m).bit_length() - 1)
    return f"{arch}|{nx}x{ny}x{nz}|fmt{vol.fmt}|lk{lookup}|m{mb}|n{n}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_shape(vol, pts, T, lookup: int, shape, reps: int = 5) -> float:
    rose.set_fitness_shape(*shape)
    rose.fitness_eval(vol, pts, T, lookup)  # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rose.fitness_eval(vol, pts, T, lookup)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(vol, pts: torch.Tensor, T: torch.Tensor, lookup: int = 0, shapes=None, cache: Optional[str] = DEFAULT_CACHE,
         force: bool = False) -> dict:
    """Pick the fastest shape for (vol, pts, T) and make it current.
    Returns {"shape": (P, U), "ms": {...}, "cached": bool}."""
    shapes = shapes or SHAPES
    key = _key(vol, pts.shape[0], T.shape[0], lookup)
    db = _load(cache) if cache else {}
    if not force and key in db and tuple(db[key]["shape"]) in shapes:
        best = tuple(db[key]["shape"])
        rose.set_fitness_shape(*best)
        return {"shape": best, "ms": db[key].get("ms", {}), "cached": True, "key": key}
    ms = {f"{p}x{u}": time_shape(vol, pts, T, lookup, (p, u)) for p, u in shapes}
    best = min(shapes, key=lambda s: ms[f"{s[0]}x{s[1]}"])
    rose.set_fitness_shape(*best)
    if cache:
        db[key] = {"shape": list(best), "ms": ms}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return {"shape": best, "ms": ms, "cached": False, "key": key}


PREFERRED = (0, 0)  # the switching mode


def tune_track(vol, depth: torch.Tensor, K, pst: torch.Tensor, params, state, shapes=None, margin: float = 0.03) -> dict:
    """Pick the fastest shape for the tracker itself: for every shape, one
    frame of pso_track_frame from a copy of `state` (the first run of each
    shape warms up), timed by the library's fitness-launch timers.  Unlike
    tune(), this measures the particles in the order the tracker schedules
    them.  A shape must beat PREFERRED by more than `margin` to replace it,
    so that near-ties (8x2 and 8x4 differ by ~2 % on one frame) resolve the
    same way in every run.  `state` is not changed.  Returns {"shape", "ms",
    "cached"}."""
    shapes = shapes or TRACK_SHAPES
    ms = {}
    rose.profile_enable(True)
    try:
        for shape in shapes:
            rose.set_fitness_shape(*shape)
            for _ in range(2):
                probe = rose.track_state(list(state.pose.q), list(state.pose.t), list(state.r))
                rose.profile_reset()
                rose.track_frame(vol, depth, K, pst, params, probe)
                prof = rose.profile_read()
            ms[f"{shape[0]}x{shape[1]}"] = prof["fitness_ms"] / max(prof["fitness_launches"], 1)
    finally:
        rose.profile_reset()
        rose.profile_enable(False)
    best = min(shapes, key=lambda sh: ms[f"{sh[0]}x{sh[1]}"])
    pk = f"{PREFERRED[0]}x{PREFERRED[1]}"
    if pk in ms and ms[f"{best[0]}x{best[1]}"] > (1.0 - margin) * ms[pk]:
        best = PREFERRED
    rose.set_fitness_shape(*best)
    return {"shape": tuple(best), "ms": ms, "cached": False}
