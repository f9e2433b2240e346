"""Smoothing kernels for svr_smooth (host-side helpers; float32 taps, unit sum).

* gauss(sigma): samples of exp(-a^2 / (2 sigma^2)) for a = -ceil(3 sigma) .. ceil(3 sigma)
  (the isotropic Gaussian of Section 4.2), normalised.
* binomial(T): row T-1 of Pascal's triangle over 2^(T-1) -- the T-tap binomial filter
  [1, 1] convolved with itself T-1 times (b_4, b_8, b_12 are the 5-, 9- and 13-tap filters).
* paper9(): the discrete 9-tap kernel behind the paper's linear-sampling 9-tap shader
  (centre weight 0.2270270270; fetches at +-1.3846153846 and +-3.2307692308 weighted
  0.3162162162 and 0.0702702703, each fetch blending its two neighbouring voxels).
* star(N): the in-ray stencil of the N-tap Gaussian (N = 5, 9, 13) in linear-sampling form,
  (c0, [(offset, weight), ...]) for svr_params star_*: binomial row N + 3 with its two
  outermost taps dropped on each side and renormalised, then neighbouring taps paired into one
  fetch each (weight w_a + w_b at offset (a w_a + b w_b) / (w_a + w_b)).  N = 9 reproduces the
  paper's printed constants; 3 (N - 1)/2 + 1 fetches per sample, the paper's count.
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


def star(N):
    if N not in (5, 9, 13):
        raise ValueError("N-tap in-ray Gaussian for N = 5, 9 or 13")
    n = N + 3
    row = np.array([math.comb(n, j) for j in range(n + 1)], dtype=np.float64)[2:-2]
    row /= row.sum()
    r = N // 2
    c0 = row[r]
    pairs = []
    for a in range(1, r + 1, 2):
        wa, wb = row[r + a], row[r + a + 1]
        pairs.append(((a * wa + (a + 1) * wb) / (wa + wb), wa + wb))
    return float(c0), [(float(o), float(w)) for o, w in pairs]
