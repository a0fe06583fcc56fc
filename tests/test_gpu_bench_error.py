"""Error against the oracle at the benchmark's stopping tolerance (1e-6 V Jacobi-scaled residual)
and at a parity tolerance, in the launch configuration bench.py times, for the workloads whose
oracle runs in seconds: the 32x32 RC grid over its 100 steps (both precisions), and the 3-layer
1024x1024 recipe at 3x256x256 over its first 300 steps (FP32 sweeps with FP64 refinement).  On
that recipe a 1e-9 V tolerance still leaves 2e-6 V (its ||M^-1 D|| is about 450), so its parity
tolerance is 1e-10 V.

The stopping test bounds each step's solve error by ||M^-1 D||_inf * tol (the oracle's
error_bound_factor), and the errors of successive steps add at most (||M^-1 C/h||_inf <= 1 for
this M-matrix), so K steps stay within K * ||M^-1 D||_inf * tol.  The measured error is printed
with that bound; the parity tolerance must meet the 1e-6 V bar."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from bench import settings
from helpers import PARITY_V, gpu_context, say
from oracle import BEStepper, mesh_to_circuit
from oracle.sources import currents_at
from oracle.spectral import error_bound_factor
from workloads import config0, config1

pytestmark = pytest.mark.gpu


def _opts(name, prec, tol):
    t = settings(name, tol, prec)
    return dict(precision=prec, tol=tol, omega=t["omega"], check_every=t["check_every"], graphs=t["graphs"],
                max_sweeps=200000, tile_rows=t["tile_rows"], scen_block=t["scen_block"],
                sweeps_per_launch=t["sweeps_per_launch"], predictor=t["predictor"])


def _max_error(w, name, prec, tol, steps):
    """max over steps 1..K and nodes of |v_gpu - v_oracle|, and the bound K ||M^-1 D|| tol."""
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    assert circ.n == mesh.n  # an RC mesh: no internal nodes
    st = BEStepper(circ, w.h)
    kappa = error_bound_factor(st.M)
    v = np.full(mesh.n, mesh.vdd)
    worst = 0.0
    with gpu_context(w, **_opts(name, prec, tol)) as ctx:
        for k in range(1, steps + 1):
            v, _ = st.step(v, np.zeros(0), currents_at(p, k * w.h))
            ctx.step(1)
            worst = max(worst, float(np.max(np.abs(ctx.read_voltages() - v))))
        stats = ctx.stats()
    bound = steps * kappa * tol
    say(f"[error] {w.name} {prec} tol={tol:g} steps={steps}: max |v - v_oracle| = {worst:.2e} V "
        f"(bound {bound:.1e} V, ||M^-1 D|| = {kappa:.2f}, {stats['sweeps'] / steps:.1f} sweeps/step)")
    return worst, bound


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_rc32_error_at_bench_and_parity_tolerance(prec):
    w = config0()
    e6, b6 = _max_error(w, "config0", prec, 1e-6, 100)
    e10, b10 = _max_error(w, "config0", prec, 1e-10, 100)
    assert e6 <= b6 and e10 <= b10
    assert e10 <= PARITY_V


@pytest.mark.timeout(900)
def test_rc3x256_error_at_bench_and_parity_tolerance():
    w = config1(side=256, steps=300)
    e6, b6 = _max_error(w, "config1", pg.PG_PREC_FP32_REFINE, 1e-6, 300)
    e10, b10 = _max_error(w, "config1", pg.PG_PREC_FP32_REFINE, 1e-10, 300)
    assert e6 <= b6 and e10 <= b10
    assert e10 <= PARITY_V
