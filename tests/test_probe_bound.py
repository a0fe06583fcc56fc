"""The rounding argument behind the opening probe's certified norm (CPU only, no device code):
the residual of a step's opening, r_i = -G0_i e_i - history_i + sum_j g_ij (e_j - e_i) with
e = v - Vdd, evaluated as the probe does in single precision (e, g and G0 rounded to FP32,
differences, products and an eight-term sum in FP32), differs from the exact value by at most
2^-19 S~_i, S~_i = G0~_i |e~_i| + sum_j g~_ij (|e~_i| + |e~_j|) accumulated in FP32.  The exact
value is computed in rational arithmetic from the FP64 inputs."""
from fractions import Fraction

import numpy as np
import pytest


def _probe_fp32(e64, g64, pad64, hist64):
    """The probe's arithmetic for one node: neighbours e64[1:] with conductances g64 (six)."""
    f = np.float32
    e = [f(x) for x in e64]
    g = [f(x) for x in g64]
    pad = f(pad64)
    e0, a0 = e[0], f(abs(e[0]))
    r = f(-pad * e0)
    s = f(pad * a0)
    for k in range(6):
        r = f(r + f(g[k] * f(e[k + 1] - e0)))
        s = f(s + f(g[k] * f(a0 + f(abs(e[k + 1])))))
    q = abs(float(r) - hist64) + float(f(f(2.0 ** -19) * s))
    return q, float(s)


def _exact(e64, g64, pad64, hist64):
    E = [Fraction(x) for x in e64]
    r = -Fraction(pad64) * E[0] - Fraction(hist64)
    for k in range(6):
        r += Fraction(g64[k]) * (E[k + 1] - E[0])
    return abs(r)


@pytest.mark.parametrize("seed", range(6))
def test_probe_norm_bounds_the_exact_residual(seed):
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(3000):
        scale = 10.0 ** rng.uniform(-9, -0.5)       # deviations from nV to ~0.3 V
        e = -scale * rng.uniform(0.0, 1.0, 7)        # drops below the supply
        if rng.uniform() < 0.3:
            e = e + scale * rng.normal(0.0, 1e-3, 7)  # nearly equal neighbours (cancellation)
        g = rng.uniform(0.5, 5.0, 6) * (rng.uniform(size=6) > 0.15)  # some edges absent
        pad = rng.choice([0.0, 10.0])
        hist = rng.normal(0.0, 1e-3) if rng.uniform() < 0.2 else 0.0
        q, s = _probe_fp32(e, g, pad, hist)
        exact = _exact(e, g, pad, hist)
        assert Fraction(q) >= exact, (e, g, pad, hist)
        # and the bound is not loose beyond its own term
        assert float(exact) >= q - 2.0 ** -18 * s - 1e-300
        worst = max(worst, (q - float(exact)) / (s + 1e-300))
    assert worst <= 2.0 ** -18


def test_rounding_term_is_needed():
    """Without the 2^-19 S term the FP32 value can fall below the exact residual: the bound is
    not vacuous."""
    rng = np.random.default_rng(7)
    below = 0
    for _ in range(3000):
        e = -0.1 * rng.uniform(0.0, 1.0, 7)
        g = rng.uniform(0.5, 5.0, 6)
        q, s = _probe_fp32(e, g, 10.0, 0.0)
        exact = _exact(e, g, 10.0, 0.0)
        below += Fraction(q - float(np.float32(np.float32(2.0 ** -19) * np.float32(s)))) < exact
    assert below > 0


def _graph_probe(v64, vref, g64, gsup64, q64, hist64, fma):
    """The netlist probe's arithmetic for one slot: v64[0] its voltage, v64[1:] its table
    entries' (padding entries carry g = 0 and the slot's own voltage), vref the reference supply,
    FP32 conductance-part values g64, the conductance to supplies and ground gsup64, and the FP64
    constant q64 and history hist64.  e_i = v_i - vref and the neighbour differences
    v_j - v_i are formed in FP64 and rounded to FP32.  With `fma` each product-accumulate rounds
    once."""
    f = np.float32
    ei = f(v64[0] - vref)
    dj = [f(x - v64[0]) for x in v64[1:]]
    g = [f(x) for x in g64]
    gs = f(gsup64)

    def acc(a, x, y):  # a + x * y in FP32
        if fma:
            return f(float(Fraction(float(a)) + Fraction(float(x)) * Fraction(float(y))))
        return f(a + f(x * y))

    r = f(-gs * ei)
    s = f(gs * f(abs(ei)))
    for k in range(len(g)):
        r = acc(r, g[k], dj[k])
        s = acc(s, g[k], f(abs(dj[k])))
    w = len(g)
    term = float(f(f(w + 8) * f(2.0 ** -23) * s))
    return abs(q64 + hist64 + float(r)) + term, float(s)


def _graph_exact(v64, vref, g64, gsup64, q64, hist64):
    V = [Fraction(x) for x in v64]
    r = Fraction(q64) + Fraction(hist64) - Fraction(gsup64) * (V[0] - Fraction(vref))
    for k in range(len(g64)):
        r += Fraction(g64[k]) * (V[k + 1] - V[0])
    return abs(r)


@pytest.mark.parametrize("fma", [False, True])
def test_netlist_probe_norm_bounds_the_exact_residual(fma):
    """The general-netlist probe: rows of 1 to 16 table entries (padding entries, zero
    conductances, near-equal neighbours, a supply term and a history, voltages around a 1.0 V
    reference and a 1.05 V second supply), evaluated with and without fused multiply-adds:
    (w + 8) 2^-23 S_i bounds the FP32 error.  The FP64 sum of the constant, the history and the
    FP32 value rounds once more at 2^-53, as the FP64 residual pass does, and the check allows
    that."""
    rng = np.random.default_rng(11 + fma)
    worst, below = 0.0, 0
    vref = 1.0
    for _ in range(4000):
        w = int(rng.integers(1, 17))
        scale = 10.0 ** rng.uniform(-9, -0.5)
        v = vref + rng.choice([0.0, 0.05]) - scale * rng.uniform(0.0, 1.0, w + 1)
        if rng.uniform() < 0.3:
            v[1:] = v[0] + scale * rng.normal(0.0, 1e-3, w)
        g = rng.uniform(0.1, 10.0, w) * (rng.uniform(size=w) > 0.2)
        pad = rng.uniform(size=w) < 0.2  # padding: g = 0 and the slot's own value
        g[pad], v[1:][pad] = 0.0, v[0]
        gsup = rng.choice([0.0, 1e-3, 10.0])
        q = rng.normal(0.0, 0.1) * gsup
        hist = rng.normal(0.0, 1e-3) if rng.uniform() < 0.2 else 0.0
        bound, s = _graph_probe(v, vref, g, gsup, q, hist, fma)
        exact = _graph_exact(v, vref, g, gsup, q, hist)
        fp64 = 2.0 ** -52 * (abs(q) + abs(hist) + float(exact))
        assert Fraction(bound) + Fraction(fp64) >= exact, (v, g, gsup, q, hist)
        term = (w + 8) * 2.0 ** -23 * s
        below += Fraction(bound - term) + Fraction(fp64) < exact  # without the term
        worst = max(worst, (float(exact) - (bound - term)) / (term + 1e-300))
    # the FP32 error uses at most the whole term, and without it the value can fall short
    assert worst <= 1.0 and below > 0
