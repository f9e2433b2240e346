"""Colour look-up tables and transfer-function control points (inputs only).

A table is an (M, 4) float32 RGBA array whose entry j sits at scalar j/(M-1); the way a
renderer reads it is not defined here.  The analytic tables are this project's own and
copy no published colour map.
"""
from __future__ import annotations

import numpy as np


def lut_ramp(m=256):
    """Grey ramp with opacity ramp: entry j = (j/(m-1)) * (1, 1, 1, 1)."""
    s = np.arange(m, dtype=np.float64) / (m - 1)
    return np.repeat(s[:, None], 4, axis=1).astype(np.float32)


def lut_heat(m=256):
    """A simple black-red-yellow-white ramp with alpha = s (piecewise linear in s)."""
    s = np.arange(m, dtype=np.float64) / (m - 1)
    r = np.clip(3 * s, 0, 1)
    g = np.clip(3 * s - 1, 0, 1)
    b = np.clip(3 * s - 2, 0, 1)
    return np.stack([r, g, b, s], axis=1).astype(np.float32)


def tf_ramp(m=64):
    """Initial transfer function: linear ramp in every channel."""
    return lut_ramp(m)


def tf_bumps(m=64, seed=1, nbumps=3):
    """Hidden target transfer function: per channel, clip(sum of 3 Gaussian bumps, 0, 1)."""
    rng = np.random.default_rng(seed)
    s = np.arange(m, dtype=np.float64) / (m - 1)
    out = np.zeros((m, 4))
    for ch in range(4):
        acc = np.zeros(m)
        for _ in range(nbumps):
            amp = rng.uniform(0.3, 1.0)
            mu = rng.uniform(0.05, 0.95)
            sig = rng.uniform(0.05, 0.25)
            acc += amp * np.exp(-((s - mu) ** 2) / (2 * sig * sig))
        out[:, ch] = np.clip(acc, 0, 1)
    return out.astype(np.float32)
