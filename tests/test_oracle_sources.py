"""Pins of the triangular current pulse (piecewise-linear source, Sec. II-A)."""
import numpy as np

from oracle.sources import triangle_current


def test_triangle_breakpoints_and_linearity():
    peak, start, width = 2e-3, 100e-12, 80e-12
    assert triangle_current(start - 1e-12, peak, start, width) == 0.0
    assert triangle_current(start, peak, start, width) == 0.0
    assert abs(triangle_current(start + 40e-12, peak, start, width) - peak) < 1e-18
    assert abs(triangle_current(start + 80e-12, peak, start, width)) < 1e-18
    assert triangle_current(start + 200e-12, peak, start, width) == 0.0
    # linear on each side: value at a quarter of the width is half the peak
    assert abs(triangle_current(start + 20e-12, peak, start, width) - peak / 2) < 1e-18
    assert abs(triangle_current(start + 60e-12, peak, start, width) - peak / 2) < 1e-18
    t = np.linspace(start, start + 40e-12, 9)
    vals = triangle_current(t, peak, start, width)
    assert np.allclose(np.diff(vals, 2), 0.0, atol=1e-15)
