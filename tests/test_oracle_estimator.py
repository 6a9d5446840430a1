"""Pins of the regrid error estimator (paper Sec. 4.5) on closed forms."""
import math

import numpy as np
import pytest


def _tile(orc, p, f):
    n = (16, 16, 1)
    t = np.zeros(orc.tile_shape(p, n))
    i = np.arange(-2, 18) + 0.5
    Y, X = np.meshgrid(i, i, indexing="ij")
    t[0, 0] = f(X, Y)
    return t, n


def test_linear_field(orc):
    """u = a + b x: |D u| = (sqrt3/2) 2 b, D^2 u = 0, so the estimate is
    bias (sqrt3/2) 2b / (|u| + eps), largest where |u| is smallest (x = -1)."""
    p = orc.make_params(ndim=2)
    a, b = 3.0, 0.1
    t, n = _tile(orc, p, lambda X, Y: a + b * X)
    e = orc.estimate(p, t, n, 0, 0, eps=1e-12, filt=0.05, bias=0.6)
    umin = a + b * (-0.5)
    assert e == pytest.approx(0.6 * math.sqrt(3) / 2 * 2 * b / (umin + 1e-12), rel=1e-13)


def test_quadratic_field_and_level_scaling(orc):
    """u = c y^2 + 5: D^2 u = 2c, |D u| = (sqrt3/2) 4 c |y|; the second-derivative
    term at y = 0.5 dominates; R^(xi (L-1)) scales the result."""
    p = orc.make_params(ndim=2)
    c = 0.01
    t, n = _tile(orc, p, lambda X, Y: c * Y * Y + 5.0)
    e1 = orc.estimate(p, t, n, 0, 0, eps=0.0, filt=0.05, bias=0.6)
    cand = []
    for y in np.arange(-1, 17) + 0.5:
        u = c * y * y + 5.0
        d1 = math.sqrt(3) / 2 * abs(c * (y + 1) ** 2 - c * (y - 1) ** 2)
        d2 = 2 * c
        cand.append(0.6 * d1 / u + 0.4 * d2 / (d1 + 0.05 * u))
    assert e1 == pytest.approx(max(cand), rel=1e-12)
    e3 = orc.estimate(p, t, n, 0, 0, eps=0.0, filt=0.05, bias=0.6, ratio=2.0, xi=-0.5, level=3)
    assert e3 == pytest.approx(e1 * 2.0 ** (-1.0), rel=1e-14)


def test_field_magnitude_mode(orc):
    """Mode 1 estimates |B|; a field of constant magnitude gives zero."""
    p = orc.make_params(ndim=2)
    n = (16, 16, 1)
    t = np.zeros(orc.tile_shape(p, n))
    i = np.arange(-2, 18) + 0.5
    Y, X = np.meshgrid(i, i, indexing="ij")
    th = 0.1 * X + 0.05 * Y
    t[4, 0] = 0.7 * np.cos(th)
    t[5, 0] = 0.7 * np.sin(th)
    assert orc.estimate(p, t, n, 1, 0, eps=0.1) < 1e-13
