"""Seeded initial parameters of the visibility surrogate MLP (inputs only).

He-uniform weights W ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases, in the
flat order W1, b1, ..., W5, b5 with W_l stored [in][out]; float32.
"""
from __future__ import annotations

import math

import numpy as np

SHAPES = [(64, 256), (256, 256), (256, 256), (256, 256), (256, 2)]


def he_uniform(seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in SHAPES:
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
