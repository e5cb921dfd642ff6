"""Pins of the oracle's Gamma variates (Marsaglia and Tsang on the Philox
streams): the distribution against scipy's Gamma law (Kolmogorov-Smirnov),
the first two moments within their standard errors, shapes below one (the
boost), the per-entry scale, and determinism of the counter layout."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("shape", [0.4, 1.0, 2.5, 31.6, 26371.1])
def test_gamma_distribution(shape):
    n = 60000
    g = philox.gamma(7, 21, shape, np.ones(n))
    ks = stats.kstest(g, stats.gamma(shape).cdf)
    assert ks.pvalue > 1e-3, ks
    assert abs(g.mean() - shape) <= 5 * np.sqrt(shape / n)
    var = g.var()
    se_var = np.sqrt((6 * shape + 2 * shape ** 2) / n)     # sd of the sample variance (excess kurtosis 6/shape)
    assert abs(var - shape) <= 5 * se_var


def test_gamma_scale_and_layout():
    sc = np.linspace(0.1, 3.0, 1000)
    a = philox.gamma(3, 5, 4.0, sc)
    b = philox.gamma(3, 5, 4.0, np.ones(1000))
    assert np.allclose(a, b * sc, rtol=1e-15)
    # element e depends only on (seed, stream, e): a prefix draws the same values
    assert np.array_equal(philox.gamma(3, 5, 4.0, np.ones(10)), b[:10])
    assert not np.array_equal(philox.gamma(3, 6, 4.0, np.ones(10)), b[:10])
