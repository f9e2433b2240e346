"""Smoothing kernels for svr_smooth (host-side helpers; float32 taps, unit sum).

* gauss(sigma): samples of exp(-a^2 / (2 sigma^2)) for a = -ceil(3 sigma) .. ceil(3 sigma)
  (the isotropic Gaussian of Section 4.2), normalised.
* binomial(T): row T-1 of Pascal's triangle over 2^(T-1) -- the T-tap binomial filter
  [1, 1] convolved with itself T-1 times (b_4, b_8, b_12 are the 5-, 9- and 13-tap filters).
* paper9(): the discrete 9-tap kernel behind the paper's linear-sampling 9-tap shader
  (centre weight 0.2270270270; fetches at +-1.3846153846 and +-3.2307692308 weighted
  0.3162162162 and 0.0702702703, each fetch blending its two neighbouring voxels).
"""
from __future__ import annotations

import math

import numpy as np


def gauss(sigma):
    r = int(math.ceil(3.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return (w / w.sum()).astype(np.float32)


def binomial(T):
    if T < 1 or T % 2 == 0:
        raise ValueError("odd tap count expected")
    n = T - 1
    w = np.array([math.comb(n, j) for j in range(T)], dtype=np.float64) / 2.0 ** n
    return w.astype(np.float32)


def paper9():
    taps = np.zeros(9)
    taps[4] = 0.2270270270
    for off, wt in ((1.3846153846, 0.3162162162), (3.2307692308, 0.0702702703)):
        i = int(off)
        f = off - i
        for side in (-1, 1):
            taps[4 + side * i] += wt * (1.0 - f)
            taps[4 + side * (i + 1)] += wt * f
    return taps.astype(np.float32)
