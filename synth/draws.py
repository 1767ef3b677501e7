"""Seeded random draws consumed by the comparison optimisers (vanilla PFO and
PSO): the optimisers take their random numbers as inputs, so that every
implementation sees the same draws."""
from __future__ import annotations

import numpy as np

PFO = 0
PSO = 1


def swarm_draws(method: int, iters: int, n: int, seed: int):
    """(draws, offsets), float32.  PFO: (iters, n, 6) standard normals and
    (iters,) uniforms in [0, 1); PSO: (iters, n, 12) uniforms in [0, 1) and
    no offsets (zeros)."""
    rng = np.random.default_rng(seed)
    if method == PFO:
        draws = rng.standard_normal((iters, n, 6), dtype=np.float32)
        offsets = rng.random(iters, dtype=np.float32)
    elif method == PSO:
        draws = rng.random((iters, n, 12), dtype=np.float32)
        offsets = np.zeros(iters, np.float32)
    else:
        raise ValueError(f"unknown method {method}")
    return draws, offsets
