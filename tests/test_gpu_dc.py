"""GPU DC operating point (pg_dc_operating_point) against the oracle's direct DC solve (eq. 3 with
A = G; inductors shorted, capacitors open), and the transient continued from it against the
oracle's backward-Euler steps from the same initial state."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import PARITY_V, compressed, gpu_context, say
from oracle import BEStepper, dc_solve, mesh_to_circuit
from oracle.sources import currents_at
from workloads import Pulses, small_multilayer, small_rc, small_rlc

pytestmark = pytest.mark.gpu


def _loads_at(p, t):
    return currents_at(p, t)


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_dc_point_of_a_loaded_three_layer_grid(prec):
    """Sources mid-pulse at t = k h: GPU DC voltages vs the oracle's DC solve, then 15 BE steps
    from that operating point vs the oracle's steps from the same state."""
    w = small_multilayer(side=45, seed=91, nl=3, pad_every=15, steps=15)
    mesh = w.meshes[0]
    k0 = 20
    p = compressed(w.pulses[0][0], start=0.2, width=2.0, peak=3.0)
    w.pulses[0][0] = p
    circ, info = mesh_to_circuit(mesh, p)
    I0 = currents_at(p, k0 * w.h)
    assert np.count_nonzero(I0) > 50
    vdc, ildc = dc_solve(circ, I0)
    say(f"[gpu] dc point 3x45x45 prec={prec}, {np.count_nonzero(I0)} loads on")
    with gpu_context(w, precision=prec, tol=1e-12, omega=1.6, max_sweeps=200000) as ctx:
        ctx.dc_operating_point(k0, omega=1.95, tol=1e-12, max_sweeps=400000)
        assert ctx.time_index() == k0
        vg = ctx.read_voltages()
        err = np.max(np.abs(vg - vdc[: mesh.n]))
        say(f"  dc err={err:.3e}, drop {1 - vdc.min():.3e} V")
        assert err <= PARITY_V and 1 - vdc.min() > 1e-3
        st = BEStepper(circ, w.h)
        v, il = vdc.copy(), ildc.copy()
        worst = 0.0
        for j in range(1, 16):
            v, il = st.step(v, il, currents_at(p, (k0 + j) * w.h))
            ctx.step(1)
            worst = max(worst, float(np.max(np.abs(ctx.read_voltages() - v[: mesh.n]))))
    say(f"  transient from the dc point: max err {worst:.3e}")
    assert worst <= PARITY_V


def test_dc_point_with_inductive_vias_and_pads():
    """Series R-L branches are their resistors at DC; the branch currents come out as
    g (v_a - v_b) and match the oracle's inductor currents (the saddle-point DC solve)."""
    w = small_rlc(side=36, seed=92, steps=10)
    mesh = w.meshes[0]
    rng = np.random.default_rng(3)
    nodes = np.sort(rng.choice(mesh.nx * mesh.ny, 300, replace=False)).astype(np.int32)
    I = rng.uniform(0, 3e-3, nodes.size)
    p = Pulses(nodes, I, np.zeros(nodes.size), np.ones(nodes.size))
    circ, info = mesh_to_circuit(mesh, p)
    vdc, ildc = dc_solve(circ, I)
    say("[gpu] dc point RLC 2x36x36")
    with gpu_context(w, precision=pg.PG_PREC_FP64, tol=1e-12, omega=1.6) as ctx:
        ctx.set_pwl(0, 0, nodes, np.arange(nodes.size + 1, dtype=np.int32), np.zeros(nodes.size), I)
        ctx.dc_operating_point(0, omega=1.9, tol=1e-13, max_sweeps=400000)
        vg, ig = ctx.read_voltages(), ctx.read_inductor_currents()
    ev = np.max(np.abs(vg - vdc[: mesh.n]))
    ei = np.max(np.abs(ig - ildc))
    say(f"  dc err v={ev:.3e} V, i={ei:.3e} A (max |i| {np.max(np.abs(ildc)):.3e})")
    assert ev <= PARITY_V
    assert ei <= 1e-6 * max(1.0, float(np.max(np.abs(ildc))))
    # KCL at the supply: the pad branches (oriented node -> supply) carry the whole load
    assert abs(np.sum(ig[mesh.via_node.size:]) + np.sum(I)) <= 1e-9 + 1e-6 * np.sum(I)


def test_dc_point_of_an_unloaded_grid_is_vdd_and_scenarios_are_independent():
    w = small_rc(40, 30, seed=93, scenarios=3, steps=1)
    mesh = w.meshes[0]
    rng = np.random.default_rng(4)
    say("[gpu] dc point, 3 scenarios (one unloaded)")
    with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-11, omega=1.6) as ctx:
        loads = []
        for s in range(3):
            nodes = np.arange(s, mesh.n, 7, dtype=np.int32)
            I = rng.uniform(0, 1e-3, nodes.size) * (s != 1)
            ctx.set_pwl(0, s, nodes, np.arange(nodes.size + 1, dtype=np.int32), np.zeros(nodes.size), I)
            loads.append((nodes, I))
        ctx.dc_operating_point(5, omega=1.9, tol=1e-12, max_sweeps=200000)
        got = [ctx.read_voltages(0, s) for s in range(3)]
    assert np.max(np.abs(got[1] - mesh.vdd)) <= 1e-12
    for s in (0, 2):
        nodes, I = loads[s]
        circ, _ = mesh_to_circuit(mesh, Pulses(nodes, I, np.zeros(nodes.size), np.ones(nodes.size)))
        vdc, _ = dc_solve(circ, I)
        assert np.max(np.abs(got[s] - vdc[: mesh.n])) <= PARITY_V


def test_dc_point_needs_a_pad_in_every_connected_part():
    """A block cut off from every pad but holding capacitance is a valid transient grid (Lemma 1)
    but has a singular DC matrix."""
    w = small_rc(24, 24, seed=94, pad_every=8, steps=1)
    mesh = w.meshes[0]
    gE = mesh.gE.reshape(1, 24, 23).copy()
    gN = mesh.gN.reshape(1, 23, 24).copy()
    gE[0, 2:6, 1] = 0.0   # cut columns around x = 2..5, rows 2..5
    gE[0, 2:6, 5] = 0.0
    gN[0, 1, 2:6] = 0.0
    gN[0, 5, 2:6] = 0.0
    mesh.gE, mesh.gN = gE, gN
    assert pg.validate_mesh(mesh)[0] == 0
    with gpu_context(w, tol=1e-10) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.dc_operating_point(0)
        assert ei.value.name == "PG_ERR_NOT_SPD"
        ctx.step(3)  # the transient is still fine
