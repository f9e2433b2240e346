"""The package's tap helpers agree with the oracle's independently written generators."""
import numpy as np

from oracle import taps as otaps
from paper_1707_00442_amd import taps as ptaps


def test_product_taps_match_oracle():
    for s in (0.7, 1.0, 2.0, 3.0):
        assert np.allclose(ptaps.gauss(s), otaps.gauss(s), rtol=0, atol=1e-7)
    for T in (3, 5, 9, 13):
        assert np.allclose(ptaps.binomial(T), otaps.binomial(T), rtol=0, atol=1e-7)
    assert np.allclose(ptaps.paper9(), otaps.paper9(), rtol=0, atol=1e-7)


def test_star_stencils_match_the_printed_constants_and_fetch_counts():
    """The in-ray N-tap stencils: N = 9 reproduces the paper's printed linear-sampling
    constants (tests/golden/paper9_taps.json, 10 printed digits); every N has unit weight
    sum and the paper's fetch count 3 (N - 1)/2 + 1 per sample (tests/golden/fetch_counts.json);
    the pairs blend to the discrete taps of their binomial row."""
    import json
    import math
    import os
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    g = json.load(open(os.path.join(gdir, "paper9_taps.json")))
    c0, pairs = ptaps.star(9)
    assert abs(c0 - g["coeff0"]) < 1e-10
    assert abs(pairs[0][0] - g["off1"]) < 1e-10 and abs(pairs[0][1] - g["coeff1"]) < 1e-10
    assert abs(pairs[1][0] - g["off2"]) < 1e-10 and abs(pairs[1][1] - g["coeff2"]) < 1e-10
    counts = json.load(open(os.path.join(gdir, "fetch_counts.json")))["gauss"]
    for N in (5, 9, 13):
        c0, pairs = ptaps.star(N)
        assert abs(c0 + 2 * sum(w for _, w in pairs) - 1.0) < 1e-12
        assert 1 + 3 * 2 * len(pairs) == counts[str(N)]
        # each pair spreads its weight over two neighbouring taps by linear interpolation;
        # the result is binomial row N + 3 without its two outermost taps per side
        taps = np.zeros(N)
        r = N // 2
        taps[r] = c0
        for o, w in pairs:
            i = int(math.floor(o))
            f = o - i
            for side in (-1, 1):
                taps[r + side * i] += w * (1 - f)
                taps[r + side * (i + 1)] += w * f
        row = np.array([math.comb(N + 3, j) for j in range(N + 4)], dtype=np.float64)[2:-2]
        assert np.max(np.abs(taps - row / row.sum())) < 1e-12
