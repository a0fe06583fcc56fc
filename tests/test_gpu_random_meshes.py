"""Randomised parity (hypothesis, fixed derandomised draws): random layered meshes of 1-4 layers
and ragged sizes, RC or with series R-L vias and pads, one to three scenarios, through the HIP
path with randomly chosen precision, tile rows and launch path (one, two or four sweeps per
launch, or the resident path where the mesh fits one workgroup), against the oracle at every node
of every step.  Bar: 1e-6 V per node per step, branch currents within 1e-6 of their largest magnitude."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_1409_7166_amd as pg
from helpers import PARITY_V, gpu_context, say
from oracle import BEStepper, mesh_to_circuit
from oracle.sources import currents_at
from oracle.transient import initial_state
from workloads import random_mesh

pytestmark = pytest.mark.gpu


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(nx=st.integers(2, 45), ny=st.integers(2, 37), nl=st.integers(1, 4), seed=st.integers(0, 10**6),
       scen=st.integers(1, 3), inductive=st.booleans(), fp32=st.booleans(), tile_rows=st.sampled_from([4, 8, 16]),
       resident=st.booleans(), spl=st.sampled_from([1, 2, 4]))
def test_random_meshes_every_node_every_step(nx, ny, nl, seed, scen, inductive, fp32, tile_rows, resident, spl):
    steps = 10
    w = random_mesh(seed, nx, ny, nl, scenarios=scen, inductive=inductive, h=1e-12 if inductive else 1e-11,
                    steps=steps)
    mesh = w.meshes[0]
    resident = resident and mesh.n <= 4096
    say(f"[gpu] random {nl}x{ny}x{nx} seed={seed} scen={scen} L={inductive} fp32={fp32} rows={tile_rows} "
        f"resident={resident} sweeps_per_launch={spl}")
    refs = []
    ind = None
    for p in w.pulses[0]:
        circ, info = mesh_to_circuit(mesh, p)
        # the oracle keeps the currents of the inductive branches only (vias, then pads); the
        # library reports every via and pad in that order, zero for the resistive ones
        ind = np.concatenate([info["internal"]["via"][0], mesh.via_node.size + info["internal"]["pad"][0]])
        st_ = BEStepper(circ, w.h)
        v, il = initial_state(circ, info, mesh.vdd)
        traj = []
        for k in range(1, steps + 1):
            v, il = st_.step(v, il, currents_at(p, k * w.h))
            traj.append((v[: mesh.n].copy(), il.copy()))
        refs.append(traj)
    prec = pg.PG_PREC_FP32_REFINE if fp32 else pg.PG_PREC_FP64
    worst_v = worst_i = 0.0
    with gpu_context(w, precision=prec, tol=1e-11, omega=1.5, check_every=8, tile_rows=tile_rows,
                     resident=int(resident), sweeps_per_launch=spl, max_sweeps=100000) as ctx:
        for k in range(steps):
            ctx.step(1)
            for s in range(scen):
                vr, ir = refs[s][k]
                worst_v = max(worst_v, float(np.max(np.abs(ctx.read_voltages(0, s) - vr))))
                if inductive and ir.size:
                    ig = ctx.read_inductor_currents(0, s)[ind]
                    worst_i = max(worst_i, float(np.max(np.abs(ig - ir))) / max(1.0, float(np.max(np.abs(ir)))))
    assert worst_v <= PARITY_V, worst_v
    assert worst_i <= 1e-6, worst_i
