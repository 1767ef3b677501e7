"""Seeded initial weights of the proposal network (inputs, not arithmetic
of the method): W ~ N(0, 2/fan_in) (He), biases 0, and the output layer
scaled by 0.01 so the initial proposal is near (mu, log-scale) = 0."""
from __future__ import annotations

import numpy as np

IN_DIM = 1216
HIDDEN = 256
OUT_DIM = 12


def init_params(seed: int, in_dim: int = IN_DIM, hidden: int = HIDDEN, out_dim: int = OUT_DIM) -> dict:
    rng = np.random.default_rng(seed)
    return {
        "W1": (rng.standard_normal((in_dim, hidden)) * np.sqrt(2.0 / in_dim)).astype(np.float32),
        "b1": np.zeros(hidden, np.float32),
        "W2": (rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)).astype(np.float32),
        "b2": np.zeros(hidden, np.float32),
        "W3": (rng.standard_normal((hidden, out_dim)) * 0.01 * np.sqrt(2.0 / hidden)).astype(np.float32),
        "b3": np.zeros(out_dim, np.float32),
    }
