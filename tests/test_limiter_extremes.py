"""The limiter factor at the extreme reconstruction increments.

The GPU q-derivative pass forms Venkatakrishnan's factor of a point and
component only at its largest positive and most negative reconstruction
increment d2, not at every neighbour: with d1 the largest (d2 > 0) or
smallest (d2 < 0) neighbour difference, min(1, ratio(d1, d2)) does not grow
with |d2| on either side, so the minimum over the neighbours is reached at
the extremes.  These checks take the minimum over every neighbour (the
oracle's form) and the two-extreme form side by side on random stencils,
including d1 = 0, eps = 0 and increments on one side only.
"""
import numpy as np
import pytest


def ratio(d1, d2, eps2):
    # the oracle's form: [(d1^2 + eps^2) d2 + 2 d2^2 d1] / [d2 (d1^2 + 2 d2^2 + d1 d2 + eps^2)]
    return ((d1 * d1 + eps2) * d2 + 2.0 * d2 * d2 * d1) / (
        d2 * (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2))


def phi_every_neighbour(d2s, dmax, dmin, eps2):
    phi = 1.0
    for d2 in d2s:
        if d2 == 0.0:
            continue
        phi = min(phi, ratio(dmax if d2 > 0 else dmin, d2, eps2))
    return max(phi, 0.0)


def phi_extremes(d2s, dmax, dmin, eps2):
    phi = 1.0
    hi, lo = max(d2s), min(d2s)
    if hi > 0:
        phi = min(phi, ratio(dmax, hi, eps2))
    if lo < 0:
        phi = min(phi, ratio(dmin, lo, eps2))
    return max(phi, 0.0)


@pytest.mark.parametrize("seed", range(6))
def test_extremes_give_the_minimum_over_neighbours(seed):
    rng = np.random.default_rng(seed)
    for _ in range(2000):
        m = int(rng.integers(1, 30))
        scale = 10.0 ** rng.uniform(-4, 1)
        d2s = rng.normal(0.0, scale, m)
        if rng.random() < 0.2:
            d2s = np.abs(d2s)            # one side only
        if rng.random() < 0.1:
            d2s[rng.integers(m)] = 0.0   # an increment of zero
        dmax = 0.0 if rng.random() < 0.1 else abs(rng.normal(0.0, scale * 2))
        dmin = 0.0 if rng.random() < 0.1 else -abs(rng.normal(0.0, scale * 2))
        eps2 = 0.0 if rng.random() < 0.1 else (scale * 10.0 ** rng.uniform(-2, 1)) ** 2
        a = phi_every_neighbour(d2s, dmax, dmin, eps2)
        b = phi_extremes(d2s, dmax, dmin, eps2)
        assert abs(a - b) <= 1e-14 * max(1.0, abs(a)), (a, b, d2s, dmax, dmin, eps2)


def test_ratio_shape():
    # >= 1 up to |d2| = |d1| / 2, then falling, on both sides
    d1, eps2 = 0.3, 1e-3
    d2 = np.linspace(1e-6, 3.0, 20001)
    f = ratio(d1, d2, eps2)
    assert np.all(f[d2 <= d1 / 2] >= 1.0 - 1e-15)
    g = f[d2 > d1 / 2]
    assert np.all(np.diff(g) <= 1e-15)
    assert np.allclose(ratio(-d1, -d2, eps2), f, rtol=1e-15, atol=0)
