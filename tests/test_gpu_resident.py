"""The resident path (pg_options.resident = 1): one workgroup per item carries whole
backward-Euler steps (right-hand side, sources, red-black sweeps, the stopping test of
Algorithm 1, the series R-L branch currents) with the voltages in LDS.  Checked against the
FP64 oracle at every node and step (RC and RLC meshes, one and three layers, scenarios on one
mesh, uneven grids up to the 4096-node limit), against the multi-launch path, for recording,
statistics, the no-convergence report and the eligibility errors."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import PARITY_V, compressed, gpu_context, oracle_run, say
from oracle import BEStepper, mesh_to_circuit
from oracle.sources import currents_at
from oracle.transient import initial_state
from workloads import Workload, config0, small_multilayer, small_rc, small_rlc

pytestmark = pytest.mark.gpu


def _opts(**kw):
    o = dict(precision=pg.PG_PREC_FP64, tol=1e-11, omega=1.6, check_every=8, resident=1, max_sweeps=100000)
    o.update(kw)
    return o


def _oracle_items(w, steps):
    """{(grid, scen): (V [steps, n], IL [steps, m])} from the oracle."""
    out = {}
    for g, (mesh, scen) in enumerate(zip(w.meshes, w.pulses)):
        for s, p in enumerate(scen):
            circ, info = mesh_to_circuit(mesh, p)
            st = BEStepper(circ, w.h)
            v, il = initial_state(circ, info, mesh.vdd)
            V, IL = [], []
            for k in range(1, steps + 1):
                v, il = st.step(v, il, currents_at(p, k * w.h))
                V.append(v[: mesh.n].copy())
                IL.append(il.copy())
            out[(g, s)] = (np.array(V), np.array(IL))
    return out


def _every_step(w, steps, **kw):
    ref = _oracle_items(w, steps)
    worst_v = worst_i = 0.0
    with gpu_context(w, **_opts(**kw)) as ctx:
        for k in range(steps):
            ctx.step(1)
            for (g, s), (V, IL) in ref.items():
                worst_v = max(worst_v, float(np.max(np.abs(ctx.read_voltages(g, s) - V[k]))))
                if IL.shape[1]:
                    il = ctx.read_inductor_currents(g, s)
                    worst_i = max(worst_i, float(np.max(np.abs(il - IL[k]))) / max(1.0, float(np.max(np.abs(IL)))))
        st = ctx.stats()
    peak = max(float(np.max(w.meshes[g].vdd - V)) for (g, s), (V, _) in ref.items())
    return worst_v, worst_i, st, peak


def test_config0_every_node_every_step():
    w = config0()
    worst, _, st, peak = _every_step(w, 100, tol=1e-10, omega=1.65, check_every=16)
    say(f"[gpu] resident 32x32: max err {worst:.3e} V, {st['sweeps'] / 100:.1f} sweeps/step, peak drop {peak:.3e} V")
    assert worst <= PARITY_V and peak > 1e-3
    assert st["steps"] == 100 and st["node_updates"] == st["sweeps"] * 1024


def test_rlc_two_layers_voltages_and_branch_currents():
    w = small_rlc(side=24, seed=51, steps=200)
    worst_v, worst_i, st, peak = _every_step(w, 200, tol=1e-12, omega=1.5)
    say(f"[gpu] resident RLC 2x24x24: err v {worst_v:.3e} V, i {worst_i:.3e} rel, peak drop {peak:.3e} V")
    assert worst_v <= PARITY_V and worst_i <= 1e-6 and peak > 1e-4


def test_three_layers_and_the_4096_node_limit():
    w = small_multilayer(side=36, seed=52, nl=3, pad_every=12, steps=40)   # 3888 nodes: two pairs per thread
    w.pulses[0][0] = compressed(w.pulses[0][0], start=0.1, width=0.5, peak=3.0)
    worst, _, st, peak = _every_step(w, 40, tol=1e-11, omega=1.7)
    say(f"[gpu] resident 3x36x36: err {worst:.3e} V, peak drop {peak:.3e} V")
    assert worst <= PARITY_V and peak > 1e-4


def test_scenarios_and_uneven_grids_in_one_launch():
    a = small_rc(40, 33, seed=53, scenarios=3, steps=60)
    b = small_rc(64, 64, seed=54, steps=60)      # 4096 nodes
    c = small_rc(17, 9, seed=55, steps=60)       # odd widths: node pairs wrap rows
    w = Workload("mixed_small", a.meshes + b.meshes + c.meshes, a.pulses + b.pulses + c.pulses, a.h, 60)
    worst, _, st, peak = _every_step(w, 60, tol=1e-11, omega=1.6)
    say(f"[gpu] resident 3 scenarios + 2 grids: err {worst:.3e} V, peak drop {peak:.3e} V")
    assert worst <= PARITY_V and peak > 1e-3


def test_matches_the_multi_launch_path_and_records():
    w = small_multilayer(side=30, seed=56, nl=2, layer_g=(1.0, 4.0), pad_every=10, steps=30)
    with gpu_context(w, **_opts(resident=0)) as ref:
        Vr = ref.run_transient(30, record_every=5)
        sr = ref.stats()
    with gpu_context(w, **_opts()) as ctx:
        V = ctx.run_transient(30, record_every=5)
        s = ctx.stats()
        assert ctx.time_index() == 30
    say(f"[gpu] resident vs multi-launch: max diff {np.max(np.abs(V - Vr)):.3e} V; sweeps {s['sweeps']} vs {sr['sweeps']}")
    assert V.shape == Vr.shape == (6, w.meshes[0].n)
    assert np.max(np.abs(V - Vr)) <= 1e-9
    assert s["steps"] == 30 and s["max_step_sweeps"] >= s["last_step_sweeps"] > 0


def test_no_convergence_is_reported_after_all_steps():
    w = config0()
    with gpu_context(w, **_opts(tol=1e-13, max_sweeps=8)) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.step(10)
        assert ei.value.name == "PG_ERR_NO_CONVERGENCE"
        assert ctx.time_index() == 10
        assert np.all(np.isfinite(ctx.read_voltages()))


def test_ineligible_grids_are_refused():
    big = small_rc(80, 52, seed=57, steps=2)     # 4160 nodes
    with gpu_context(big, **_opts()) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.step(1)
        assert ei.value.name == "PG_ERR_UNSUPPORTED"
    w = config0()
    with gpu_context(w, **_opts(ordering=pg.PG_ORDER_JACOBI)) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.step(1)
        assert ei.value.name == "PG_ERR_UNSUPPORTED"


def test_enqueued_steps_captured_in_a_hip_graph_and_replayed():
    """pg_step_enqueue captured once on the context's stream and replayed four times, with eager
    work and synchronisations between the replays: after each replay the state equals, bit for
    bit, that of a context stepped eagerly to the same step; the clock and statistics follow."""
    import torch
    a = small_rc(40, 33, seed=58, scenarios=3, steps=60)
    b = small_rc(24, 20, seed=59, steps=60)
    w = Workload("graph_small", a.meshes + b.meshes, a.pulses + b.pulses, a.h, 60)
    items = [(0, 0), (0, 1), (0, 2), (1, 0)]
    torch.cuda.set_device(0)
    side = torch.cuda.Stream()
    ctx = pg.Context(0, side.cuda_stream)
    ctx.set_options(h=w.h, tol=1e-11, omega=1.6, check_every=8, precision=pg.PG_PREC_FP64, resident=1,
                    max_sweeps=100000)
    for g, (mesh, scen) in enumerate(zip(w.meshes, w.pulses)):
        ctx.upload_mesh(mesh, len(scen))
        for s, p in enumerate(scen):
            ctx.set_pulses(g, s, p)
    with gpu_context(w, **_opts()) as ref:
        with ctx:
            ctx.step(2)          # builds the coefficients (allocates) outside the capture
            ref.step(2)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=side):
                ctx.step_enqueue(5)
            torch.cuda.synchronize()
            done = 2             # capture queues nothing
            for r in range(4):
                graph.replay()
                x = torch.ones(1 << 20, device="cuda:0").sum()   # eager work between the replays
                torch.cuda.synchronize()
                done += 5
                ref.step(5)
                assert ctx.time_index() == done == ref.time_index()
                for it in items:
                    assert np.array_equal(ctx.read_voltages(*it), ref.read_voltages(*it)), (r, it)
                assert float(x) == float(1 << 20)
            st, sr = ctx.stats(), ref.stats()
            say(f"[gpu] graph replay of enqueued resident steps: {done} steps, sweeps {st['sweeps']} vs {sr['sweeps']}")
            assert st["sweeps"] == sr["sweeps"] and st["node_updates"] == sr["node_updates"]
            ctx.step(3)          # eager steps continue from the replayed state
            ref.step(3)
            for it in items:
                assert np.array_equal(ctx.read_voltages(*it), ref.read_voltages(*it))
            with pytest.raises(pg.PgError):
                ctx.set_options(resident=0)
                ctx.step_enqueue(1)
