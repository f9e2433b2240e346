"""Smoothing kernels of Section 4.2 (test infrastructure; plain definitions).

* ``binomial(T)``: the T-tap binomial filter b_{T-1} = [1, 1]^{*(T-1)} (cascaded
  autoconvolution of [1, 1]), normalised to unit sum.  The paper names b_4, b_8, b_12 the
  5-, 9- and 13-tap filters.
* ``paper9()``: the discrete 9-tap kernel equivalent to the paper's linear-sampling
  9-tap shader (one centre fetch and two fetches per side at fractional offsets, each a
  linear blend of two neighbouring voxels).
* ``gauss(sigma)``: exp(-a^2 / 2 sigma^2) sampled at a = -ceil(3 sigma) .. ceil(3 sigma),
  normalised to unit sum (Eq. Gaussian, isotropic).
"""
from __future__ import annotations

import math

import numpy as np

# Section 4.2, Alg. 9-tap Gaussian smoothing: centre weight, two (offset, weight) pairs.
PAPER9_CENTRE_WEIGHT = 0.2270270270
PAPER9_PAIRS = ((1.3846153846, 0.3162162162), (3.2307692308, 0.0702702703))


def binomial(T):
    if T < 1 or T % 2 == 0:
        raise ValueError("binomial filters have an odd tap count")
    b = np.array([1.0])
    for _ in range(T - 1):
        b = np.convolve(b, [1.0, 1.0])
    return b / b.sum()


def linear_sampling_to_taps(centre_weight, pairs):
    """Expand (offset, weight) fetch pairs with linear interpolation into discrete taps.

    A fetch at fractional offset o = i + f (i integer) with weight w reads
    (1 - f) V[i] + f V[i+1], i.e. adds w (1 - f) to tap i and w f to tap i + 1, on both
    sides of the centre.
    """
    reach = max(int(math.floor(o)) + 1 for o, _ in pairs)
    taps = np.zeros(2 * reach + 1)
    c = reach
    taps[c] += centre_weight
    for o, w in pairs:
        i = int(math.floor(o))
        f = o - i
        for sgn in (1, -1):
            taps[c + sgn * i] += w * (1 - f)
            taps[c + sgn * (i + 1)] += w * f
    return taps


def paper9():
    return linear_sampling_to_taps(PAPER9_CENTRE_WEIGHT, PAPER9_PAIRS)


def gauss(sigma):
    r = int(math.ceil(3.0 * sigma))
    a = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(a * a) / (2.0 * sigma * sigma))
    return g / g.sum()


def fwhm(sigma):
    """Eq. FWHM: full width at half maximum of a Gaussian of standard deviation sigma."""
    return 2.0 * math.sqrt(2.0 * math.log(2.0)) * sigma
