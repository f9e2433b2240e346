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
