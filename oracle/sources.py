"""Current-source waveforms (test infrastructure only).

The paper models device currents as piecewise-linear ideal current sources
(Sec. II-A).  The workloads use one symmetric triangle per source: zero
outside [start, start + width], peak at the midpoint.

Parity: pinned by ``tests/test_oracle_sources.py`` (breakpoint values and
linearity between breakpoints).
"""
from __future__ import annotations

import numpy as np


def triangle_current(t: float, peak, start, width) -> np.ndarray:
    """i(t) = peak * max(0, 1 - |t - (start + width/2)| / (width/2))."""
    half = 0.5 * np.asarray(width, float)
    mid = np.asarray(start, float) + half
    return np.asarray(peak, float) * np.maximum(0.0, 1.0 - np.abs(t - mid) / half)


def currents_at(pulses, t: float) -> np.ndarray:
    """Current of every source branch (pulse order) at time t."""
    if pulses is None or pulses.count == 0:
        return np.zeros(0)
    return triangle_current(t, pulses.peak, pulses.start, pulses.width)
