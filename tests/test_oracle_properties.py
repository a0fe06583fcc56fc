"""Property tests of the oracle on random layered meshes (hypothesis): for any shape, value draw
and load pattern, a backward-Euler step (eq. 2; eq. 10 with series R-L vias and pads) keeps
Kirchhoff's current law summed over the grid, never lifts a node above the supply under
non-negative loads (the step matrix is an M-matrix, so its inverse is non-negative), is linear
in the loads, and leaves the scaled residual of its own solution at rounding level."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import BEStepper, BESystem, mesh_to_circuit, scaled_residual
from oracle.sources import currents_at
from oracle.transient import initial_state
from workloads import Pulses, random_mesh

SHAPES = dict(nx=st.integers(2, 9), ny=st.integers(2, 9), nl=st.integers(1, 3), seed=st.integers(0, 10**6))
SETTINGS = settings(max_examples=40, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


def _run(w, pulses, steps):
    mesh = w.meshes[0]
    circ, info = mesh_to_circuit(mesh, pulses)
    st_ = BEStepper(circ, w.h)
    v, il = initial_state(circ, info, mesh.vdd)
    out = []
    for k in range(1, steps + 1):
        v, il = st_.step(v, il, currents_at(pulses, k * w.h))
        out.append((v.copy(), il.copy()))
    return circ, info, out


@SETTINGS
@given(**SHAPES)
def test_rc_charge_balance_and_maximum_principle(nx, ny, nl, seed):
    w = random_mesh(seed, nx, ny, nl, steps=8)
    mesh, p = w.meshes[0], w.pulses[0][0]
    _, _, out = _run(w, p, 8)
    C = mesh.C.ravel()
    prev = np.full(mesh.n, mesh.vdd)
    for k, (v, _) in enumerate(out, start=1):
        vm = v[: mesh.n]
        I = currents_at(p, k * w.h).sum()
        q = np.sum(C / w.h * (vm - prev))
        pad = np.sum(mesh.pad_g * (vm[mesh.pad_node] - mesh.vdd))
        assert abs(q + pad + I) <= 1e-11 * max(1.0, abs(I), float(np.sum(C / w.h)))
        assert np.all(vm <= mesh.vdd + 1e-13)
        prev = vm


@SETTINGS
@given(inductive=st.booleans(), **SHAPES)
def test_linearity_in_the_loads(nx, ny, nl, seed, inductive):
    w = random_mesh(seed, nx, ny, nl, inductive=inductive, h=1e-12 if inductive else 1e-11, steps=6)
    mesh, p = w.meshes[0], w.pulses[0][0]
    half = np.arange(p.count) % 2 == 0
    a = Pulses(p.node, np.where(half, p.peak, 0.0), p.start, p.width)
    b = Pulses(p.node, np.where(half, 0.0, p.peak), p.start, p.width)
    _, _, va = _run(w, a, 6)
    _, _, vb = _run(w, b, 6)
    _, _, vab = _run(w, p, 6)
    for (x, ix), (y, iy), (z, iz) in zip(va, vb, vab):
        # drops below the supply add; so do the branch currents
        assert np.max(np.abs((mesh.vdd - x) + (mesh.vdd - y) - (mesh.vdd - z))) <= 1e-12
        if ix.size:
            assert np.max(np.abs(ix + iy - iz)) <= 1e-12 * max(1.0, float(np.max(np.abs(iz))))


@SETTINGS
@given(inductive=st.booleans(), **SHAPES)
def test_the_step_solution_has_a_rounding_level_residual(nx, ny, nl, seed, inductive):
    w = random_mesh(seed, nx, ny, nl, inductive=inductive, h=1e-12 if inductive else 1e-11, steps=3)
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info, out = _run(w, p, 3)
    sysm = BESystem(circ, w.h)
    v0, il0 = initial_state(circ, info, mesh.vdd)
    prev = (v0, il0)
    for k, (v, il) in enumerate(out, start=1):
        res = scaled_residual(sysm, prev[0], prev[1], v, currents_at(p, k * w.h))
        assert res <= 1e-13
        # a perturbation of one node by delta shows up as about delta
        vp = v.copy()
        vp[len(vp) // 2] += 1e-6
        assert scaled_residual(sysm, prev[0], prev[1], vp, currents_at(p, k * w.h)) >= 0.5e-6
        prev = (v, il)
