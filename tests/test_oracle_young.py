"""Pins of the oracle's recursive Gaussian (Young and van Vliet 1995, the O(1)
convolution the paper uses for Gaussian windows, Sec. II-C).

The published method fixes: unit DC gain (B = 1 - (b1 + b2 + b3) / b0 makes
each pass sum to 1 on an unbounded signal), an impulse response symmetric
about the impulse (a causal pass followed by the same anti-causal pass), and
a shape close to the sampled Gaussian of the requested sigma (its q(sigma)
fit).  A mistyped coefficient breaks the last (a swapped digit in one of the
six polynomial constants moves the RMS error from 0.25 % to 1..30 % of the
peak).  The filter's second moment is about 1.2 sigma^2 (its tails decay more
slowly than the Gaussian's), which is a property of the 1995 design, checked
loosely here.
"""
import numpy as np
import pytest

import oracle


def _impulse(sigma, N=2001):
    c = N // 2
    d = np.zeros((N, 1))
    d[c] = 1.0
    r = oracle.young_1d(d, sigma, 0)[:, 0]
    j = np.arange(N) - c
    return r, j, c


@pytest.mark.parametrize("sigma", [0.8, 1.0, 2.0, 2.6, 3.0, 5.0, 10.0])
def test_young_impulse_response(sigma):
    r, j, c = _impulse(sigma)
    assert abs(r.sum() - 1.0) < 1e-9
    assert np.abs(r[c + 1:] - r[c - 1::-1][:len(r) - c - 1]).max() < 1e-12
    g = np.exp(-j ** 2 / (2.0 * sigma ** 2))
    g /= g.sum()
    assert np.sqrt(((r - g) ** 2).mean()) / g.max() < 0.005
    var = (r * j * j).sum()
    assert 1.1 * sigma ** 2 < var < 1.7 * sigma ** 2


def test_young_separable_and_linear():
    """young_conv filters rows then columns: the same as the transposed order
    (the passes are linear and act on different axes), and linear in u."""
    rng = np.random.default_rng(2)
    u = rng.random((2, 23, 31))
    v = rng.random((2, 23, 31))
    a = oracle.young_conv(u, 2.5)
    b = oracle.young_1d(oracle.young_1d(u, 2.5, 1), 2.5, 2)
    assert np.abs(a - b).max() < 1e-13
    assert np.abs(oracle.young_conv(2.0 * u - v, 2.5) - (2.0 * a - oracle.young_conv(v, 2.5))).max() < 1e-13


def test_young_fast_filter_constant_image():
    """Any linear window: a constant image is returned unchanged."""
    f = np.full((3, 20, 27), 0.37)
    g = np.random.default_rng(1).random((3, 20, 27))
    cen = oracle.bisecting_kmeans(g, 6).centers
    P, _, _ = oracle.pinv(oracle.kernel_matrix(cen, 0.3))
    out, _ = oracle.fast_filter(f, g, cen, P, 2.0, 0.3, spatial="young")
    assert np.abs(out - 0.37).max() < 1e-12
