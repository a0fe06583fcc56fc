"""The smallest shapes the boundary accepts, against the oracle at every node of every step:
2x2 meshes, two-wide strips in either direction, a 2x2 stack of three and four layers joined
through every node, and a one-node netlist.  They exercise the tiles' padding columns and rows,
the red ring at every edge of a grid that fits in one workgroup, and the opening probe (the
steps after the pulses converge at once).  Meshes narrower than two nodes are refused at upload
(the netlist path takes them), which the last test checks."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import PARITY_V, compressed, gpu_context, oracle_run, say
from oracle import BEStepper, Circuit, GROUND
from oracle.sources import currents_at
from workloads import Pulses, Workload, small_multilayer, small_rc

pytestmark = pytest.mark.gpu

STEPS = 40


def _cases():
    out = [small_rc(2, 2, seed=61, steps=STEPS), small_rc(2, 37, seed=62, steps=STEPS),
           small_rc(37, 2, seed=63, steps=STEPS), small_rc(3, 3, seed=64, steps=STEPS)]
    for nl, layer_g in ((3, (1.0, 2.0, 4.0)), (4, (1.0, 2.0, 3.0, 4.0))):
        out.append(small_multilayer(side=2, seed=64 + nl, nl=nl, layer_g=layer_g, via_every=1, pad_every=1,
                                    fraction=1.0, steps=STEPS))
    return out


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_smallest_meshes_every_node_every_step(prec):
    worst_all = 0.0
    for w in _cases():
        mesh = w.meshes[0]
        p = compressed(w.pulses[0][0], start=0.1, width=0.4, peak=3.0)
        w2 = Workload(w.name, [mesh], [[p]], w.h, STEPS)
        Vref, _ = oracle_run(mesh, p, w.h, STEPS)
        with gpu_context(w2, precision=prec, tol=1e-12, omega=1.2) as ctx:
            V = ctx.run_transient(STEPS)
            st = ctx.stats()
        err = float(np.max(np.abs(V - Vref)))
        say(f"[gpu] {w.name} {mesh.nx}x{mesh.ny}x{mesh.nl} prec={prec}: err={err:.2e} V, "
            f"drop={float(np.max(mesh.vdd - Vref)):.2e} V, sweeps={st['sweeps']}")
        assert err <= PARITY_V
        assert float(np.max(mesh.vdd - Vref)) > 1e-4  # the pulses act
        worst_all = max(worst_all, err)
    assert worst_all <= PARITY_V


def test_one_node_netlist():
    """One node with a capacitor, a pad to a 1.1 V supply and a load: each step is the scalar
    recurrence v' = ((C/h) v + g Vs - I) / (C/h + g)."""
    C, g, vs, h = 2e-12, 4.0, 1.1, 1e-11
    frm = np.array([0, 0, 0], np.int32)
    to = np.array([GROUND, 1, GROUND], np.int32)
    kind = np.array(list("CRI"))
    val = np.array([C, g, 0.0])
    p = Pulses(np.array([0], np.int32), np.array([5e-3]), np.array([1e-11]), np.array([2e-10]))
    circ = Circuit(1, np.array([vs]), frm.astype(np.int64), to.astype(np.int64), kind, val)
    st = BEStepper(circ, h)
    ctx = pg.Context(0)
    with ctx:
        ctx.set_options(h=h, tol=1e-13, omega=1.0, check_every=2, precision=pg.PG_PREC_FP64)
        gid = ctx.upload_netlist(1, 1, [vs], frm, to, kind, val, None, 1)
        ctx.set_pulses(gid, 0, p)
        v, x = np.array([vs]), vs
        worst = 0.0
        for k in range(1, 31):
            I = currents_at(p, k * h)
            v, _ = st.step(v, np.zeros(0), I)
            x = ((C / h) * x + g * vs - I[0]) / (C / h + g)
            ctx.step(1)
            got = float(ctx.read_voltages(gid)[0])
            assert abs(v[0] - x) < 1e-14
            worst = max(worst, abs(got - x))
    say(f"[gpu] one-node netlist: err={worst:.2e} V")
    assert worst <= 1e-9


def test_meshes_narrower_than_two_nodes_are_refused():
    w = small_rc(1, 40, seed=65, steps=2)
    with pg.Context(0) as ctx:
        with pytest.raises(pg.PgError) as e:
            ctx.upload_mesh(w.meshes[0], 1)
    assert e.value.status == -1
