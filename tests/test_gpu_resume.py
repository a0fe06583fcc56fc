"""Bitwise resume: a transient of K steps gives the same bits as k steps, a read of the state
(voltages and inductor currents of every scenario), a fresh context set to that state and clock
(pg_set_state, pg_set_time), and K - k more steps.  Algorithm 1 warm-starts each step from the
previous step's solution V(s-1) and nothing else, so the state and the clock are the whole
input of the remaining run.  The resume point lies inside the current pulses, where every step
sweeps, so the resumed steps take the same decisions as the uninterrupted ones."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import gpu_context, say, torch_stream
from workloads import irregular_grid, small_multilayer, small_rc, small_rlc

pytestmark = pytest.mark.gpu

K, k_resume = 60, 25


def _mesh_case(name):
    if name == "rc3":
        return small_multilayer(side=96, seed=31, nl=3, pad_every=16, steps=K)
    if name == "rlc2":
        return small_rlc(side=64, seed=32, steps=K)
    return small_rc(48, 40, seed=33, scenarios=3, steps=K)


def _items(ctx, w):
    return [(g, s) for g in range(len(w.pulses)) for s in range(len(w.pulses[g]))]


def _state(ctx, items):
    return {it: (ctx.read_voltages(*it), ctx.read_inductor_currents(*it)) for it in items}


@pytest.mark.parametrize("name,prec", [("rc3", pg.PG_PREC_FP32_REFINE), ("rlc2", pg.PG_PREC_FP64),
                                       ("rlc2", pg.PG_PREC_FP32_REFINE), ("batch", pg.PG_PREC_FP32_REFINE)])
def test_mesh_resume_is_bitwise(name, prec):
    w = _mesh_case(name)
    opts = dict(precision=prec, tol=1e-10, omega=1.6, check_every=8)
    say(f"[gpu] resume {name} prec={prec}: {K} steps vs {k_resume} + set_state + {K - k_resume}")
    with gpu_context(w, **opts) as a:
        items = _items(a, w)
        a.step(K)
        full = _state(a, items)
        # the same context: reset, k steps, read, reset, restore, the rest
        a.reset()
        a.step(k_resume)
        mid = _state(a, items)
        a.reset()
        for it, (v, il) in mid.items():
            a.set_state(*it, v, il)
        a.set_time_index(k_resume)
        a.step(K - k_resume)
        again = _state(a, items)
    with gpu_context(w, **opts) as b:
        for it, (v, il) in mid.items():
            b.set_state(*it, v, il)
        b.set_time_index(k_resume)
        b.step(K - k_resume)
        resumed = _state(b, items)
    for it in items:
        assert np.array_equal(full[it][0], resumed[it][0]), it
        assert np.array_equal(full[it][1], resumed[it][1]), it
        assert np.array_equal(full[it][0], again[it][0]), it
        assert np.array_equal(full[it][1], again[it][1]), it
    assert max(float(np.max(1.0 - full[it][0])) for it in items) > 1e-4  # a loaded state


def test_netlist_resume_is_bitwise():
    net, scen = irregular_grid(side=24, nl=2, seed=34, rlc=True, scenarios=2)
    say(f"[gpu] resume general netlist n={net.n}")

    def ctx():
        c = pg.Context(0, torch_stream())
        c.set_options(h=10e-12, tol=1e-10, omega=1.6, check_every=8, precision=pg.PG_PREC_FP32_REFINE)
        g = c.upload_netlist(net.n, net.p, net.source_v, net.frm, net.to, net.kind, net.value, None, len(scen))
        for s, p in enumerate(scen):
            c.set_pulses(g, s, p)
        return c

    items = [(0, s) for s in range(len(scen))]
    with ctx() as a:
        a.step(K)
        full = _state(a, items)
    with ctx() as a:
        a.step(k_resume)
        mid = _state(a, items)
    with ctx() as b:
        for it, (v, il) in mid.items():
            b.set_state(*it, v, il)
        b.set_time_index(k_resume)
        b.step(K - k_resume)
        resumed = _state(b, items)
    for it in items:
        assert np.array_equal(full[it][0], resumed[it][0]), it
        assert np.array_equal(full[it][1], resumed[it][1]), it
    assert np.max(np.abs(full[(0, 0)][1])) > 0  # inductor currents flow
