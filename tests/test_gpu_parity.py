"""GPU parity: the HIP transient (through the C ABI) against the FP64 oracle.

Bar: max |v_gpu - v_oracle| <= 1e-6 V for every node and every step, at a stopping
tolerance tight enough for that bar (the tolerance-to-error relation is stated per test).
"""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import PARITY_V, compressed, gpu_context, oracle_run, say, torch_stream
from oracle import BEStepper, dc_solve, mesh_to_circuit
from workloads import Pulses, config0, small_multilayer, small_rc, small_rlc

pytestmark = pytest.mark.gpu


def _run_and_compare(w, steps, **opts):
    mesh, p = w.meshes[0], w.pulses[0][0]
    say(f"[gpu] {w.name} steps={steps} opts={opts}")
    with gpu_context(w, **opts) as ctx:
        V = ctx.run_transient(steps)
        st = ctx.stats()
    Vref, _ = oracle_run(mesh, p, w.h, steps)
    err = np.max(np.abs(V - Vref), axis=1)
    say(f"  sweeps={st['sweeps']} max_step_sweeps={st['max_step_sweeps']} "
        f"max_err={err.max():.3e} V final_res={st['last_residual']:.2e}")
    return err, st, V, Vref


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_config0_parity_every_node_every_step(prec):
    w = config0()
    err, st, V, Vref = _run_and_compare(w, 100, precision=prec, tol=1e-10, omega=1.6)
    assert err.max() <= PARITY_V
    assert st["steps"] == 100 and st["sweeps"] > 0
    assert np.max(1.0 - Vref) > 1e-3  # the pulses produce a real drop


def test_config0_jacobi_ordering_same_fixed_point():
    w = config0()
    err, st, _, _ = _run_and_compare(w, 60, ordering=pg.PG_ORDER_JACOBI, omega=0.9, tol=1e-10,
                                     max_sweeps=20000)
    assert err.max() <= PARITY_V


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_three_layer_ragged_parity(prec):
    """3 layers, 100 x 100 (ragged against 64-wide, 16-row tiles), vias every 4, pads every 32."""
    w = small_multilayer(side=100, seed=31, nl=3, pad_every=32, steps=60)
    w.pulses[0][0] = compressed(w.pulses[0][0], start=0.08, width=1.0)
    err, st, _, _ = _run_and_compare(w, 60, precision=prec, tol=1e-11, omega=1.8, check_every=16)
    assert err.max() <= PARITY_V


@pytest.mark.parametrize("rows", [4, 16])
def test_tile_rows_do_not_change_the_result(rows):
    w = small_multilayer(side=90, seed=32, nl=2, pad_every=30, steps=30)
    w.pulses[0][0] = compressed(w.pulses[0][0], start=0.05, width=1.0)
    err, _, _, _ = _run_and_compare(w, 30, tile_rows=rows, tol=1e-11, omega=1.7)
    assert err.max() <= PARITY_V


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_rlc_ragged_parity_voltages_and_currents(prec):
    """Series R-L vias and pads (eq. 10): node voltages and branch currents every step."""
    w = small_rlc(side=70, seed=33, steps=150)
    mesh = w.meshes[0]
    p = compressed(w.pulses[0][0], start=0.2, width=0.5, peak=2.0)
    w.pulses[0][0] = p
    steps = 150
    say(f"[gpu] rlc 2x70x70 prec={prec}")
    circ, info = mesh_to_circuit(mesh, p)
    st = BEStepper(circ, w.h)
    from oracle.transient import initial_state
    from oracle.sources import currents_at
    v, il = initial_state(circ, info, mesh.vdd)
    worst_v = worst_i = 0.0
    with gpu_context(w, precision=prec, tol=1e-12, omega=1.9, check_every=16, max_sweeps=50000) as ctx:
        for k in range(1, steps + 1):
            v, il = st.step(v, il, currents_at(p, k * w.h))
            ctx.step(1)
            vg = ctx.read_voltages()
            ig = ctx.read_inductor_currents()
            worst_v = max(worst_v, float(np.max(np.abs(vg - v[: mesh.n]))))
            worst_i = max(worst_i, float(np.max(np.abs(ig - il))))
        stats = ctx.stats()
    say(f"  sweeps={stats['sweeps']} max_err_v={worst_v:.3e} V max_err_i={worst_i:.3e} A")
    assert worst_v <= PARITY_V
    assert worst_i <= 1e-6 * max(1.0, float(np.max(np.abs(il))))
    assert np.max(np.abs(il)) > 1e-5


def test_zero_current_stays_at_vdd():
    w = small_multilayer(side=80, seed=34, nl=3, pad_every=16, steps=20)
    p = w.pulses[0][0]
    w.pulses[0][0] = Pulses(p.node, np.zeros_like(p.peak), p.start, p.width)
    say("[gpu] zero current")
    with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-12) as ctx:
        V = ctx.run_transient(20)
    assert np.max(np.abs(V - 1.0)) <= 1e-12


def test_dc_steady_state_matches_direct_solve():
    """Constant sources and a long step: the transient settles on the DC point (eq. 3, A = G)."""
    w = small_rc(48, 40, seed=35, steps=1)
    mesh = w.meshes[0]
    rng = np.random.default_rng(7)
    nodes = np.arange(0, mesh.n, 3, dtype=np.int32)
    I = rng.uniform(0, 2e-3, nodes.size)
    say("[gpu] dc steady state")
    with gpu_context(w, h=1e-9, tol=1e-12, omega=1.9, max_sweeps=200000) as ctx:
        ctx.set_pwl(0, 0, nodes, np.arange(nodes.size + 1, dtype=np.int32), np.zeros(nodes.size), I)
        ctx.step(400)
        vg = ctx.read_voltages()
    p = Pulses(nodes, I, np.zeros(nodes.size), np.ones(nodes.size))
    circ, info = mesh_to_circuit(mesh, p)
    vdc, _ = dc_solve(circ, I)
    err = np.max(np.abs(vg - vdc[: mesh.n]))
    say(f"  dc err={err:.3e}")
    assert err <= PARITY_V
    assert np.max(1.0 - vdc) > 1e-3


def test_bitwise_deterministic():
    w = small_multilayer(side=96, seed=36, nl=3, pad_every=32, steps=25)
    w.pulses[0][0] = compressed(w.pulses[0][0], start=0.05, width=1.0)
    say("[gpu] determinism")
    runs = []
    for _ in range(2):
        with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-9, omega=1.8) as ctx:
            runs.append(ctx.run_transient(25))
    assert np.array_equal(runs[0], runs[1])


def test_no_convergence_reported_and_state_kept():
    w = config0()
    say("[gpu] no convergence")
    with gpu_context(w, tol=1e-14, max_sweeps=2, check_every=1) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.step(50)
        assert ei.value.name == "PG_ERR_NO_CONVERGENCE"
        assert ctx.time_index() == 50
        v = ctx.read_voltages()
        assert np.all(np.isfinite(v)) and np.max(1.0 - v) > 0


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_batched_scenarios_share_one_mesh(prec):
    """Six current scenarios on one 70 x 44 mesh in one context: every scenario against its own
    oracle transient, and scenarios converge independently (per-item masks)."""
    base = small_rc(70, 44, seed=41, scenarios=6, steps=40)
    mesh = base.meshes[0]
    scen = [compressed(p, start=0.4, width=1.0) for p in base.pulses[0]]
    scen[3] = Pulses(scen[3].node, np.zeros_like(scen[3].peak), scen[3].start, scen[3].width)
    base.pulses[0] = scen
    say(f"[gpu] 6 scenarios prec={prec}")
    with gpu_context(base, precision=prec, tol=1e-11, omega=1.6) as ctx:
        ctx.step(40)
        got = [ctx.read_voltages(0, s) for s in range(6)]
    for s, p in enumerate(scen):
        Vref, _ = oracle_run(mesh, p, base.h, 40)
        err = np.max(np.abs(got[s] - Vref[-1]))
        say(f"  scenario {s}: err={err:.3e}")
        assert err <= PARITY_V
    assert np.max(np.abs(got[3] - 1.0)) <= 1e-12


@pytest.mark.parametrize("prec,ordering,rows,block,nl", [
    (pg.PG_PREC_FP64, pg.PG_ORDER_RED_BLACK, 4, 3, 4),
    (pg.PG_PREC_FP32_REFINE, pg.PG_ORDER_RED_BLACK, 16, 2, 3),
    (pg.PG_PREC_FP32_REFINE, pg.PG_ORDER_RED_BLACK, 8, 16, 2),
    (pg.PG_PREC_FP64, pg.PG_ORDER_JACOBI, 8, 4, 2),
])
def test_scenario_blocks_on_layered_meshes(prec, ordering, rows, block, nl):
    """Five scenarios on one layered 77 x 77 mesh, swept in scenario blocks (ragged blocks,
    blocks larger than the batch, every layer count's ring tasks), each against its own oracle."""
    lg = (1.0, 2.0, 4.0, 8.0)[:nl]
    w = small_multilayer(side=77, seed=81, nl=nl, layer_g=lg, pad_every=16, steps=25)
    w.pulses[0] = [compressed(small_multilayer(side=77, seed=90 + s, nl=nl, layer_g=lg, pad_every=16).pulses[0][0],
                              start=0.25, width=1.0) for s in range(5)]
    say(f"[gpu] scenario blocks prec={prec} ordering={ordering} rows={rows} block={block} nl={nl}")
    omega = 0.9 if ordering == pg.PG_ORDER_JACOBI else 1.6
    with gpu_context(w, precision=prec, tol=1e-11, omega=omega, tile_rows=rows, scen_block=block,
                     ordering=ordering, max_sweeps=20000) as ctx:
        ctx.step(25)
        got = [ctx.read_voltages(0, s) for s in range(5)]
    for s, p in enumerate(w.pulses[0]):
        Vref, _ = oracle_run(w.meshes[0], p, w.h, 25)
        err = np.max(np.abs(got[s] - Vref[-1]))
        say(f"  scenario {s}: err={err:.3e}")
        assert err <= PARITY_V


@pytest.mark.parametrize("case", ["rc32_fp64", "three_layer_fp32", "blocks_fp32", "four_layer_fp64",
                                  "rlc_fp32_rows8", "four_layer_fp32", "blocks_fp64"])
def test_two_sweeps_per_launch_equal_two_launches(case):
    """Fusing two red-black sweeps into one launch gives the voltages of two separate sweeps bit
    for bit, including an odd cycle length (one single-sweep launch at the end of each cycle),
    ragged tiles and scenario blocks: where the tile shape has the kernel the tile is staged with
    a four-node halo once (three_layer_fp32, rlc_fp32_rows8, four_layer_fp32, blocks_fp32 and
    blocks_fp64 scenario by scenario, and the one-layer FP64 rc32_fp64), else the halo's rings are
    recomputed (four_layer_fp64)."""
    lg4 = (1.0, 2.0, 4.0, 8.0)
    if case == "rc32_fp64":
        w, prec, rows, chk, block = config0(), pg.PG_PREC_FP64, 8, 7, 0
    elif case == "three_layer_fp32":
        w, prec, rows, chk, block = (small_multilayer(side=100, seed=31, nl=3, pad_every=32, steps=20),
                                     pg.PG_PREC_FP32_REFINE, 16, 8, 0)
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.08, width=1.0)
    elif case == "blocks_fp32":
        w = small_multilayer(side=77, seed=81, nl=2, layer_g=lg4[:2], pad_every=16, steps=20)
        w.pulses[0] = [compressed(small_multilayer(side=77, seed=90 + s, nl=2, layer_g=lg4[:2],
                                                   pad_every=16).pulses[0][0], start=0.25, width=1.0)
                       for s in range(5)]
        prec, rows, chk, block = pg.PG_PREC_FP32_REFINE, 4, 5, 3
    elif case == "four_layer_fp64":
        w = small_multilayer(side=77, seed=82, nl=4, layer_g=lg4, pad_every=16, steps=20)
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.25, width=1.0)
        prec, rows, chk, block = pg.PG_PREC_FP64, 4, 9, 0
    elif case == "four_layer_fp32":
        w = small_multilayer(side=77, seed=84, nl=4, layer_g=lg4, pad_every=16, steps=20)
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.25, width=1.0)
        prec, rows, chk, block = pg.PG_PREC_FP32_REFINE, 4, 9, 0
    elif case == "blocks_fp64":
        w = small_multilayer(side=140, seed=85, nl=1, layer_g=lg4[:1], pad_every=16, steps=20)
        w.pulses[0] = [compressed(small_multilayer(side=140, seed=95 + s, nl=1, layer_g=lg4[:1],
                                                   pad_every=16).pulses[0][0], start=0.25, width=1.0)
                       for s in range(5)]
        prec, rows, chk, block = pg.PG_PREC_FP64, 8, 5, 2
    else:
        w = small_rlc(side=150, seed=83, steps=20)
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.02, width=0.3)
        prec, rows, chk, block = pg.PG_PREC_FP32_REFINE, 8, 7, 0
    steps = 20
    res = {}
    for spl in (1, 2):
        say(f"[gpu] fused sweeps case={case} sweeps_per_launch={spl}")
        with gpu_context(w, precision=prec, tol=1e-11, omega=1.6, tile_rows=rows, check_every=chk,
                         scen_block=block, sweeps_per_launch=spl) as ctx:
            ctx.step(steps)
            res[spl] = ([ctx.read_voltages(0, s) for s in range(len(w.pulses[0]))], ctx.stats())
            staged = case in ("three_layer_fp32", "rlc_fp32_rows8", "blocks_fp32", "rc32_fp64", "four_layer_fp32",
                              "blocks_fp64")
            assert ctx.sweep_launch_info() == ((2, staged) if spl == 2 else (1, False))
    for a, b in zip(res[1][0], res[2][0]):
        assert np.array_equal(a, b), np.max(np.abs(a - b))
    assert res[1][1]["sweeps"] == res[2][1]["sweeps"]
    Vref, _ = oracle_run(w.meshes[0], w.pulses[0][0], w.h, steps)
    err = np.max(np.abs(res[2][0][0] - Vref[-1]))
    say(f"  sweeps={res[2][1]['sweeps']} err={err:.3e}")
    assert err <= PARITY_V


@pytest.mark.parametrize("case", ["rlc_two_layer_rows8", "one_layer_rows16", "two_layer_rows4", "ragged_rows4",
                                  "blocks_rows16", "one_layer_fp64_rows8", "unsupported_falls_back"])
def test_four_sweeps_per_launch_equal_four_launches(case):
    """Four red-black sweeps per launch (temporal blocking: the tile with an 8-node halo staged
    once, four sweeps on chip) give the voltages of four separate sweeps bit for bit: several
    tiles in x and y so the halos overlap neighbouring tiles, ragged edges, cycle lengths that
    leave one-sweep launches at the end of a cycle, the RLC grid's branch currents, scenario
    blocks, FP64 sweeps, and a context whose tile groups have no four-sweep kernel (it sweeps
    once per launch)."""
    lg4 = (1.0, 2.0, 4.0, 8.0)
    if case == "rlc_two_layer_rows8":
        w, rows, chk = small_rlc(side=300, seed=71, steps=30), 8, 16
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.02, width=0.3)
    elif case == "one_layer_rows16":
        w, rows, chk = small_multilayer(side=260, seed=72, nl=1, layer_g=lg4[:1], pad_every=16, steps=20), 16, 10
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.25, width=1.0)
    elif case == "two_layer_rows4":
        w, rows, chk = small_multilayer(side=140, seed=73, nl=2, layer_g=lg4[:2], pad_every=32, steps=20), 4, 9
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.08, width=1.0)
    elif case == "ragged_rows4":
        w, rows, chk = small_multilayer(side=77, seed=74, nl=2, layer_g=lg4[:2], pad_every=16, steps=20), 4, 7
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.25, width=1.0)
    elif case == "blocks_rows16":  # five scenarios on one mesh, swept in blocks of three
        w, rows, chk = small_multilayer(side=150, seed=76, nl=1, layer_g=lg4[:1], pad_every=16, steps=20), 16, 10
        w.pulses[0] = [compressed(small_multilayer(side=150, seed=96 + s, nl=1, layer_g=lg4[:1],
                                                   pad_every=16).pulses[0][0], start=0.25, width=1.0)
                       for s in range(5)]
    elif case == "one_layer_fp64_rows8":
        w, rows, chk = small_multilayer(side=200, seed=77, nl=1, layer_g=lg4[:1], pad_every=16, steps=20), 8, 12
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.25, width=1.0)
    else:  # three layers: no four-sweep kernel for that shape
        w, rows, chk = small_multilayer(side=100, seed=75, nl=3, pad_every=32, steps=20), 4, 8
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.08, width=1.0)
    steps = w.steps if w.steps <= 30 else 30
    res = {}
    ns = len(w.pulses[0])
    for spl in (1, 4):
        say(f"[gpu] four sweeps per launch case={case} sweeps_per_launch={spl}")
        prec = pg.PG_PREC_FP64 if "fp64" in case else pg.PG_PREC_FP32_REFINE
        with gpu_context(w, precision=prec, tol=1e-11, omega=1.6, tile_rows=rows,
                         check_every=chk, sweeps_per_launch=spl, scen_block=3, max_sweeps=50000) as ctx:
            ctx.step(steps)
            res[spl] = ([ctx.read_voltages(0, s) for s in range(ns)],
                        [ctx.read_inductor_currents(0, s) for s in range(ns)], ctx.stats())
            fused = (4, True) if case != "unsupported_falls_back" else (1, False)
            assert ctx.sweep_launch_info() == (fused if spl == 4 else (1, False))
    for s in range(ns):
        assert np.array_equal(res[1][0][s], res[4][0][s]), np.max(np.abs(res[1][0][s] - res[4][0][s]))
        assert np.array_equal(res[1][1][s], res[4][1][s])
    assert res[1][2]["sweeps"] == res[4][2]["sweeps"]
    Vref, _ = oracle_run(w.meshes[0], w.pulses[0][0], w.h, steps)
    err = np.max(np.abs(res[4][0][0] - Vref[-1]))
    say(f"  sweeps={res[4][2]['sweeps']} err={err:.3e}")
    assert err <= PARITY_V


def test_netlist_upload_equals_mesh_upload():
    """An RLC grid uploaded as the oracle's branch list (pg_upload_netlist) steps bit for bit like
    the same grid uploaded as a mesh, and both match the oracle."""
    w = small_rlc(side=40, seed=61, steps=25)
    mesh = w.meshes[0]
    p = compressed(w.pulses[0][0], start=0.02, width=0.2)
    w.pulses[0][0] = p
    circ, _ = mesh_to_circuit(mesh, p)
    say("[gpu] netlist upload vs mesh upload (RLC 2x40x40)")
    opts = dict(precision=pg.PG_PREC_FP64, tol=1e-11, omega=1.6)
    with gpu_context(w, **opts) as ctx:
        ctx.step(25)
        v_mesh, i_mesh = ctx.read_voltages(), ctx.read_inductor_currents()
    ctx = pg.Context(0, torch_stream())
    base = dict(h=w.h, check_every=8)
    base.update(opts)
    ctx.set_options(**base)
    with ctx:
        gid = ctx.upload_netlist(circ.n, circ.p, circ.vd, circ.frm, circ.to, circ.kind, circ.value,
                                 (mesh.nx, mesh.ny, mesh.nl))
        ctx.set_pulses(gid, 0, p)
        ctx.step(25)
        v_net, i_net = ctx.read_voltages(), ctx.read_inductor_currents()
    assert np.array_equal(v_mesh, v_net) and np.array_equal(i_mesh, i_net)
    Vref, _ = oracle_run(mesh, p, w.h, 25)
    assert np.max(np.abs(v_net - Vref[-1])) <= PARITY_V


@pytest.mark.parametrize("graphs", [0, 1])
def test_queued_openings_change_nothing(graphs):
    """pg_step(n) queues each step's close and the next step's opening before the step's last
    decision (and backs off when the step needs more sweeps); stepping one call per step never
    does.  Both give the same voltages bit for bit and the same sweep counts, on a batch whose
    steps alternate between converging at once and needing several cycles."""
    w = small_rc(70, 44, seed=43, scenarios=3, steps=60)
    w.pulses[0] = [compressed(p, start=0.5, width=1.0) for p in w.pulses[0]]
    res = []
    for mode in ("one call", "per step"):
        say(f"[gpu] queued openings graphs={graphs} mode={mode}")
        with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-9, omega=1.6, graphs=graphs) as ctx:
            if mode == "one call":
                ctx.step(60)
            else:
                for _ in range(60):
                    ctx.step(1)
            res.append(([ctx.read_voltages(0, s) for s in range(3)], ctx.stats(), ctx.time_index()))
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    assert res[0][1]["sweeps"] == res[1][1]["sweeps"] and res[0][1]["steps"] == res[1][1]["steps"] == 60
    assert res[0][2] == res[1][2] == 60


def test_uneven_grids_batched_in_one_launch():
    """Three grids of different sizes and layer counts stepped together in one context."""
    ws = [small_rc(33, 70, seed=51, steps=30), small_multilayer(side=77, seed=52, nl=2, pad_every=16, steps=30),
          small_rc(130, 9, seed=53, steps=30)]
    from workloads import Workload
    w = Workload("mixed", [x.meshes[0] for x in ws], [[compressed(x.pulses[0][0], start=0.3, width=1.0)] for x in ws],
                 ws[0].h, 30)
    say("[gpu] 3 uneven grids")
    with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-11, omega=1.6) as ctx:
        ctx.step(30)
        got = [ctx.read_voltages(g, 0) for g in range(3)]
        st = ctx.stats()
    for g in range(3):
        Vref, _ = oracle_run(w.meshes[g], w.pulses[g][0], w.h, 30)
        err = np.max(np.abs(got[g] - Vref[-1]))
        say(f"  grid {g}: err={err:.3e}")
        assert err <= PARITY_V
    assert st["node_updates"] > 0


@pytest.mark.parametrize("case", ["rc32", "three_layer", "batched"])
def test_graph_replay_matches_eager_every_step(case):
    """Replaying the captured step graphs gives bitwise the eager launches' voltages after every
    step (host reads and synchronisations happen between replays)."""
    if case == "rc32":
        w, prec = config0(), pg.PG_PREC_FP64
    elif case == "three_layer":
        w, prec = small_multilayer(side=100, seed=71, nl=3, pad_every=32, steps=30), pg.PG_PREC_FP32_REFINE
        w.pulses[0][0] = compressed(w.pulses[0][0], start=0.08, width=1.0)
    else:
        w, prec = small_rc(70, 44, seed=72, scenarios=4, steps=30), pg.PG_PREC_FP32_REFINE
        w.pulses[0] = [compressed(p, start=0.4, width=1.0) for p in w.pulses[0]]
    steps = 30
    out = {}
    for graphs in (0, 1):
        say(f"[gpu] graphs={graphs} case={case}")
        with gpu_context(w, precision=prec, tol=1e-10, omega=1.6, graphs=graphs) as ctx:
            V = []
            for k in range(steps):
                ctx.step(1)
                V.append(np.stack([ctx.read_voltages(0, s) for s in range(len(w.pulses[0]))]))
            out[graphs] = (np.array(V), ctx.stats())
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1]["sweeps"] == out[1][1]["sweeps"]
    assert out[0][1]["node_updates"] == out[1][1]["node_updates"]


def test_autotune_restores_state_and_caches(tmp_path):
    w = small_multilayer(side=96, seed=81, nl=2, pad_every=32, steps=20)
    w.pulses[0][0] = compressed(w.pulses[0][0], start=0.05, width=1.0)
    cache = str(tmp_path / "tune.json")
    say("[gpu] autotune")
    with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-10, omega=1.0) as ctx:
        ctx.step(5)
        v5 = ctx.read_voltages()
        chosen = ctx.autotune(4, cache)
        assert ctx.time_index() == 5
        assert np.array_equal(ctx.read_voltages(), v5)
        assert 0 < chosen["omega"] < 2 and chosen["check_every"] >= 1 and chosen["tile_rows"] in (4, 8, 16)
        assert chosen["sweeps_per_launch"] in (1, 2, 4)
        ctx.step(15)
        V = ctx.read_voltages()
    import json
    entry = list(json.load(open(cache)).values())[0]
    assert entry["omega"] == pytest.approx(chosen["omega"])
    Vref, _ = oracle_run(w.meshes[0], w.pulses[0][0], w.h, 20)
    assert np.max(np.abs(V - Vref[-1])) <= PARITY_V
    with gpu_context(w, precision=pg.PG_PREC_FP32_REFINE, tol=1e-10, omega=1.0) as ctx:
        again = ctx.autotune(4, cache)
    assert again["omega"] == pytest.approx(chosen["omega"]) and again["check_every"] == chosen["check_every"]
    assert again["sweeps_per_launch"] == chosen["sweeps_per_launch"] and again["tile_rows"] == chosen["tile_rows"]


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_probe_opening_that_finds_work(prec):
    """A grid with no sources converges at once, so its next openings only take the norm (the
    right-hand side is formed inside that pass); a state set from outside then makes such an
    opening find work, and its b and r are stored before the first sweep.  Every step against
    the oracle from the same state."""
    w = small_multilayer(side=48, seed=37, nl=2, pad_every=16, steps=12)
    mesh = w.meshes[0]
    rng = np.random.default_rng(11)
    v_pert = mesh.vdd - rng.uniform(0.0, 0.02, mesh.n)
    circ, info = mesh_to_circuit(mesh, None)
    st = BEStepper(circ, w.h)
    say(f"[gpu] probe opening prec={prec}")
    with gpu_context(w, precision=prec, tol=1e-11, omega=1.6) as ctx:
        ctx.set_pulses(0, 0, Pulses(np.zeros(0, np.int32), np.zeros(0), np.zeros(0), np.zeros(0)))
        ctx.step(3)  # converged at once: the later openings are probes
        assert np.max(np.abs(ctx.read_voltages() - mesh.vdd)) <= 1e-12
        ctx.set_state(0, 0, v_pert)
        v = v_pert.copy()
        worst = 0.0
        for k in range(10):
            v, _ = st.step(v, np.zeros(0), np.zeros(0))
            ctx.step(1)
            worst = max(worst, float(np.max(np.abs(ctx.read_voltages() - v))))
        stats = ctx.stats()
    say(f"  max err={worst:.3e} V, sweeps={stats['sweeps']}")
    assert worst <= PARITY_V and stats["sweeps"] > 0


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_probe_norm_bounds_the_fp64_residual(prec):
    """An opening predicted to converge at once takes the FP32 probe, whose norm must bound the
    FP64 Jacobi-scaled residual from above and exceed it by at most its rounding term,
    2^-19 max_i S_i / M_ii with S_i = sum_j |M_ij| (|e_i| + |e_j|) (e = v - Vdd): a state whose
    residual sits below the tolerance is accepted unchanged with that norm, and one above it is
    stepped."""
    from oracle import BESystem, scaled_residual
    w = small_multilayer(side=40, seed=43, nl=3, pad_every=8, steps=4)
    mesh = w.meshes[0]
    circ, info = mesh_to_circuit(mesh, None)
    sysm = BESystem(circ, w.h)
    rng = np.random.default_rng(17)
    delta = rng.uniform(0.0, 1.0, mesh.n)
    none = np.zeros(0)
    unit = scaled_residual(sysm, mesh.vdd - delta, none, mesh.vdd - delta, none)  # linear in delta
    tol = 1e-6
    A = abs(sysm.M.tocsr())
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    for target, quiet in ((0.3 * tol, True), (3.0 * tol, False)):
        vq = mesh.vdd - delta * (target / unit)
        true = scaled_residual(sysm, vq, none, vq, none)
        e = np.abs(vq - mesh.vdd)
        # sum_j |M_ij| |e_j| + (sum_j |M_ij|) |e_i| covers S_i (M_ii >= G0_i + sum_j g_ij)
        slack = 2.0 ** -19 * float(np.max((A @ e + rowsum * e) / sysm.M.diagonal()))
        say(f"[gpu] probe bound prec={prec} target={target:.1e} true={true:.3e} slack={slack:.1e}")
        with gpu_context(w, precision=prec, tol=tol, omega=1.6) as ctx:
            ctx.set_pulses(0, 0, Pulses(np.zeros(0, np.int32), np.zeros(0), np.zeros(0), np.zeros(0)))
            ctx.step(2)  # converged at once from v = Vdd: the next opening is a probe
            ctx.set_state(0, 0, vq)
            ctx.step(1)
            st = ctx.stats()
            v1 = ctx.read_voltages()
        if quiet:
            say(f"  accepted: probe norm={st['last_residual']:.6e}")
            assert st["last_step_sweeps"] == 0 and np.array_equal(v1, vq)
            assert true <= st["last_residual"] <= true * (1 + 1e-9) + slack
        else:
            assert st["last_step_sweeps"] > 0 and st["last_residual"] <= tol
