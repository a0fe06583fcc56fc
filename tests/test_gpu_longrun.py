"""Whole-length parity of the benchmarked workloads against the FP64 oracle, every step.

* The 3-layer recipe of the benchmarked mesh at a reduced size: every node of every one of its
  1000 steps (the oracle runs in a worker process beside the GPU).
* The full 3-layer 1024 x 1024 mesh: at every one of its 1000 steps, the voltages of a seeded
  sample of nodes and the largest drop over all nodes against the oracle values stored in
  ``tests/golden/`` (``make_golden.py``), and the oracle-assembled FP64 residual of sampled steps.
* The 256-scenario batch: every node of every scenario at every one of its 500 steps.
* The 64 uneven grids: every node of every grid at every 5th of their 500 steps.
* The RLC mesh: every node and every branch current at every 5th of its first 500 steps.
* The adjoint workload over all 200 steps: the loss, sampled gradient entries against the oracle
  adjoint and a directional derivative against a central difference of the oracle's transient.

All runs use the launch configuration ``bench.py`` times (its tuned omega, sweeps per check, tile
rows and scenario blocks) at the parity tolerance ``bench.PARITY_TOL``.  The bar is the 1e-6 V
per-node, per-step bar; branch currents are held to 1e-6 of their largest magnitude."""
import os

import numpy as np
import pytest
import torch

import paper_1409_7166_amd as pg
from bench import GOLDEN, PARITY_TOL, settings
from helpers import PARITY_V, gpu_context, say
from oracle_stream import BatchStream, OracleStream, balanced_chunks
from workloads import config1, config2, config3a, config3b

pytestmark = pytest.mark.gpu

WORKERS = 16  # CPU share of one GPU on the test boxes


def _opts(name, prec):
    tol = PARITY_TOL[name]
    t = settings(name, tol, prec)
    return dict(precision=prec, tol=tol, omega=t["omega"], check_every=t["check_every"], graphs=t["graphs"],
                max_sweeps=200000, tile_rows=t["tile_rows"], scen_block=t["scen_block"],
                sweeps_per_launch=t["sweeps_per_launch"], predictor=t["predictor"])


def _read_all(ctx, w, bufs):
    """Voltages of every (grid, scenario) item, gathered on the device and copied once."""
    for (g, s), b in bufs.items():
        ctx.read_voltages_dev(g, s, b)
    return {it: b.cpu().numpy() for it, b in bufs.items()}


def _bufs(w, items):
    return {(g, s): torch.empty(w.meshes[g].n, dtype=torch.float64, device="cuda:0") for g, s in items}


@pytest.mark.timeout(900)
def test_config1_recipe_every_node_every_step():
    side = int(os.environ.get("PG_TEST_PROXY_SIDE", "320"))
    w = config1(side=side, steps=1000)
    mesh = w.meshes[0]
    say(f"[gpu] 3x{side}x{side} (the 3-layer 1024x1024 recipe), 1000 steps, every node vs oracle")
    stream = OracleStream("mesh_trajectory", (("config1", {"side": side, "steps": 1000}), [(0, 0)], 1000), 8)
    worst, worst_k, peak = 0.0, 0, 0.0
    try:
        with gpu_context(w, **_opts("config1", pg.PG_PREC_FP32_REFINE)) as ctx:
            buf = _bufs(w, [(0, 0)])
            for k in range(1, 1001):
                ctx.step(1)
                got = _read_all(ctx, w, buf)[(0, 0)]
                kk, vs, _ = stream.get()
                assert kk == k
                e = float(np.max(np.abs(got - vs[0])))
                if e > worst:
                    worst, worst_k = e, k
                peak = max(peak, float(mesh.vdd - vs[0].min()))
                if k % 100 == 0:
                    say(f"  step {k}: max error so far {worst:.3e} V (step {worst_k})")
            st = ctx.stats()
    finally:
        stream.close()
    say(f"  {st['sweeps'] / 1000:.1f} sweeps/step; max |v - v_oracle| = {worst:.3e} V at step {worst_k}; "
        f"peak drop {peak:.3e} V")
    assert worst <= PARITY_V
    assert peak > 1e-3


@pytest.mark.timeout(900)
def test_config1_full_size_sampled_nodes_every_step():
    path = GOLDEN["config1"]
    if not os.path.exists(path):
        pytest.skip("stored oracle values for the 3x1024x1024 mesh are missing (tests/golden/make_golden.py)")
    g = np.load(path)
    nodes, ref, ref_max = g["nodes"], g["drops"].astype(np.float64), g["max_drop"]
    steps = int(g["steps"])
    w = config1(steps=steps)
    mesh = w.meshes[0]
    vdd = mesh.vdd
    say(f"[gpu] 3x1024x1024, {steps} steps, {nodes.size} sampled nodes and the largest drop vs oracle")
    buf = torch.empty(mesh.n, dtype=torch.float64, device="cuda:0")
    idx = torch.from_numpy(nodes.astype(np.int64)).to("cuda:0")
    worst = worst_max = 0.0
    with gpu_context(w, **_opts("config1", pg.PG_PREC_FP32_REFINE)) as ctx:
        for k in range(steps):
            ctx.step(1)
            ctx.read_voltages_dev(0, 0, buf)
            d = vdd - buf
            samp = d[idx].cpu().numpy()
            worst = max(worst, float(np.max(np.abs(samp - ref[k]))))
            worst_max = max(worst_max, abs(float(d.max()) - float(ref_max[k])))
            if (k + 1) % 200 == 0:
                say(f"  step {k + 1}: sampled error {worst:.3e} V, largest-drop error {worst_max:.3e} V")
        st = ctx.stats()
    say(f"  {st['sweeps'] / steps:.1f} sweeps/step; peak drop {ref_max.max():.3e} V")
    # float32 storage of the drops (<= 0.06 V) adds at most 0.06 * 2^-24 = 4e-9 V
    assert worst <= PARITY_V and worst_max <= PARITY_V
    assert ref_max.max() > 1e-3


@pytest.mark.timeout(900)
def test_config3a_every_scenario_every_step():
    w = config3a()
    S, steps = len(w.pulses[0]), w.steps
    items = [(0, s) for s in range(S)]
    say(f"[gpu] {S} scenarios x 256x256, {steps} steps, every node of every scenario vs oracle")
    chunks = balanced_chunks(items, [1.0] * S, WORKERS)
    worst = np.zeros(S)
    with BatchStream(("config3a", {}), chunks, steps) as bs:
        with gpu_context(w, **_opts("config3a", pg.PG_PREC_FP32_REFINE)) as ctx:
            bufs = _bufs(w, items)
            for k in range(1, steps + 1):
                ctx.step(1)
                got = _read_all(ctx, w, bufs)
                kk, ref, _ = bs.get()
                assert kk == k
                for s in range(S):
                    worst[s] = max(worst[s], float(np.max(np.abs(got[(0, s)] - ref[(0, s)]))))
                if k % 100 == 0:
                    say(f"  step {k}: max error so far {worst.max():.3e} V (scenario {int(worst.argmax())})")
            st = ctx.stats()
    say(f"  {st['sweeps'] / steps:.1f} scenario-sweeps/step; max error {worst.max():.3e} V")
    assert worst.max() <= PARITY_V


@pytest.mark.timeout(900)
def test_config3b_every_grid_every_5th_step():
    w = config3b()
    G, steps, every = len(w.meshes), w.steps, 5
    items = [(g, 0) for g in range(G)]
    n = np.array([m.n for m in w.meshes], float)
    say(f"[gpu] {G} uneven grids ({int(n.sum()):,} nodes), {steps} steps, every node of every grid "
        f"at every {every}th step vs oracle")
    chunks = balanced_chunks(items, n * np.log2(n), WORKERS)
    worst = np.zeros(G)
    with BatchStream(("config3b", {}), chunks, steps, every) as bs:
        with gpu_context(w, **_opts("config3b", pg.PG_PREC_FP32_REFINE)) as ctx:
            bufs = _bufs(w, items)
            for k in range(every, steps + 1, every):
                ctx.step(every)
                got = _read_all(ctx, w, bufs)
                kk, ref, _ = bs.get()
                assert kk == k
                for g in range(G):
                    worst[g] = max(worst[g], float(np.max(np.abs(got[(g, 0)] - ref[(g, 0)]))))
                if k % 100 == 0:
                    say(f"  step {k}: max error so far {worst.max():.3e} V (grid {int(worst.argmax())})")
    say(f"  max error {worst.max():.3e} V")
    assert worst.max() <= PARITY_V


@pytest.mark.timeout(900)
def test_config2_rlc_every_5th_step_of_500():
    steps, every = 500, 5
    w = config2(steps=steps)
    mesh = w.meshes[0]
    say(f"[gpu] RLC 2x512x512, {steps} steps, every node and branch current at every {every}th step")
    stream = OracleStream("mesh_trajectory", (("config2", {"steps": steps}), [(0, 0)], steps, every, True), 8)
    worst_v = worst_i = imax = 0.0
    try:
        with gpu_context(w, **_opts("config2", pg.PG_PREC_FP32_REFINE)) as ctx:
            buf = _bufs(w, [(0, 0)])
            for k in range(every, steps + 1, every):
                ctx.step(every)
                got = _read_all(ctx, w, buf)[(0, 0)]
                il_gpu = ctx.read_inductor_currents()
                kk, vs, ils = stream.get()
                assert kk == k
                worst_v = max(worst_v, float(np.max(np.abs(got - vs[0]))))
                worst_i = max(worst_i, float(np.max(np.abs(il_gpu - ils[0]))))
                imax = max(imax, float(np.max(np.abs(ils[0]))))
                if k % 100 == 0:
                    say(f"  step {k}: max error v {worst_v:.3e} V, i {worst_i:.3e} A")
    finally:
        stream.close()
    say(f"  max |i| {imax:.3e} A")
    assert worst_v <= PARITY_V
    assert worst_i <= 1e-6 * max(1.0, imax)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("launch", ["fp32_one_sweep", "bench_fp64_four_sweeps"])
def test_config4_adjoint_all_200_steps(launch):
    """The adjoint workload over its whole 200 steps with checkpoints every 20: the loss, seeded
    sampled entries of every gradient against the oracle adjoint (per entry within 1e-4 of the
    larger of the entry and 1e-3 of the gradient's largest magnitude), and the directional
    derivative along a seeded direction against a central difference of the oracle's forward
    transient on the full grid (within 1e-4 relative); with FP32 sweeps one per launch, and with
    the settings bench.py times (FP64 sweeps four per launch on 16-row tiles, each solve started
    from the extrapolated iterate)."""
    from workloads import config4, random_direction
    path = os.path.join(os.path.dirname(GOLDEN["config1"]), "config4_adjoint_samples.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle adjoint values are missing (tests/golden/make_golden.py config4_adjoint)")
    g = np.load(path)
    w = config4()
    mesh = w.meshes[0]
    steps, margin = int(g["steps"]), float(g["margin"])
    say(f"[gpu] adjoint 1024x1024, {steps} steps, checkpoints every 20, {launch}")
    if launch == "fp32_one_sweep":
        opts = dict(precision=pg.PG_PREC_FP32_REFINE, tol=1e-11, omega=1.5, max_sweeps=100000)
    else:
        t = settings("config4", 1e-10, pg.PG_PREC_FP64)
        opts = dict(precision=pg.PG_PREC_FP64, tol=1e-10, omega=t["omega"], check_every=t["check_every"],
                    tile_rows=t["tile_rows"], sweeps_per_launch=t["sweeps_per_launch"], max_sweeps=100000,
                    predictor=t["predictor"])
    with gpu_context(w, **opts) as ctx:
        J = ctx.loss_forward(0, 0, steps, 20, margin)
        dC, dE, dN = ctx.loss_backward(1e-10)
        if launch != "fp32_one_sweep":
            assert ctx.sweep_launch_info() == (4, True)
    worst = 0.0
    for name, grad in (("C", dC), ("gE", dE), ("gN", dN)):
        ref = g[f"grad_{name}"]
        got = grad.ravel()[g[f"idx_{name}"]]
        floor = 1e-3 * float(g[f"maxabs_{name}"])
        err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
        worst = max(worst, float(err.max()))
    d = random_direction(mesh)
    dot = float(np.sum(dC * d[0]) + np.sum(dE * d[1]) + np.sum(dN * d[2]))
    fd, dot_ref = float(g["dir_fd"]), float(g["dir_dot"])
    say(f"  J={J:.10e} (oracle {float(g['J']):.10e}); worst sampled gradient error {worst:.2e}; "
        f"directional {dot:.8e}, oracle adjoint {dot_ref:.8e}, oracle central difference {fd:.8e}")
    assert abs(J - float(g["J"])) <= 1e-9 * abs(float(g["J"]))
    assert worst <= 1e-4
    assert abs(dot - fd) <= 1e-4 * abs(fd)
