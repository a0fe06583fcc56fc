"""GPU estimates of the Jacobi spectral radius (Young's omega) and of the residual-to-error
factor ||M^-1 D||_inf, against closed forms and the oracle, and the adaptive tolerance they
give: a step stopped at tol = err / kappa is within err of the exact backward-Euler step."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import compressed, gpu_context, say
from oracle import BESystem, BEStepper, error_bound_factor, jacobi_radius, mesh_to_circuit, young_omega
from oracle.sources import currents_at
from workloads import small_multilayer, small_rc, uniform_diagonal_mesh

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_rho_and_kappa_of_the_uniform_diagonal_grid(prec):
    nx = ny = 24
    g, C, h = 1.0, 2e-12, 1e-11
    w = uniform_diagonal_mesh(nx, ny, g=g, C=C, h=h)
    rho_exact = g * 4 * np.cos(np.pi / (nx + 1)) / (C / h + 4 * g)
    circ, _ = mesh_to_circuit(w.meshes[0], None)
    kappa_ref = error_bound_factor(BESystem(circ, h).M)
    say(f"[gpu] uniform-diagonal 24x24 prec={prec}: rho {rho_exact:.6f}, kappa {kappa_ref:.4f}")
    with gpu_context(w, precision=prec, tol=1e-10, omega=1.5) as ctx:
        rho, omega = ctx.estimate_omega(0, iters=1024)
        kappa = ctx.error_bound_factor(0, rel_tol=1e-10)
    say(f"  gpu rho {rho:.6f} omega {omega:.5f} kappa {kappa:.6f}")
    assert rho == pytest.approx(rho_exact, rel=1e-4)
    assert omega == pytest.approx(young_omega(rho_exact), rel=1e-3)
    assert kappa == pytest.approx(kappa_ref, rel=1e-7)


def test_rho_of_step_and_dc_matrices_of_a_layered_grid():
    w = small_multilayer(side=30, seed=21, nl=2, layer_g=(1.0, 2.0), pad_every=10)
    mesh = w.meshes[0]
    circ, _ = mesh_to_circuit(mesh, None)
    ref_step = jacobi_radius(BESystem(circ, w.h).M)
    ref_dc = jacobi_radius(circ.matrices()["G"])
    say(f"[gpu] rho 2x30x30: step {ref_step:.6f}, dc {ref_dc:.6f}")
    with gpu_context(w, precision=pg.PG_PREC_FP64, tol=1e-10) as ctx:
        v0 = ctx.read_voltages()
        rho_s, _ = ctx.estimate_omega(0, dc=False, iters=2048)
        rho_d, w_d = ctx.estimate_omega(0, dc=True, iters=8192)
        assert np.array_equal(ctx.read_voltages(), v0)
        ctx.step(2)  # the step matrix is back after the DC estimate
    say(f"  gpu step {rho_s:.6f} dc {rho_d:.6f} (omega {w_d:.4f})")
    assert rho_s == pytest.approx(ref_step, rel=1e-4)
    assert rho_d == pytest.approx(ref_dc, rel=1e-3)


def test_adaptive_tolerance_bounds_a_step_error():
    """From the oracle's exact state, one GPU step stopped at tol = err / kappa lies within err of
    the oracle's exact next state (and a tolerance 30x looser is measurably less accurate)."""
    w = small_rc(64, 48, seed=22, pad_every=16, steps=30)
    mesh = w.meshes[0]
    p = compressed(w.pulses[0][0], start=0.3, width=1.0, peak=2.0)
    w.pulses[0][0] = p
    circ, info = mesh_to_circuit(mesh, p)
    st = BEStepper(circ, w.h)
    v = np.full(circ.n, mesh.vdd)
    il = np.zeros(0)
    k0 = 12
    for k in range(1, k0 + 1):
        v, il = st.step(v, il, currents_at(p, k * w.h))
    v_next, _ = st.step(v, il, currents_at(p, (k0 + 1) * w.h))
    err = 1e-7
    say("[gpu] adaptive tolerance, rc 64x48")
    with gpu_context(w, precision=pg.PG_PREC_FP64, tol=1e-6, omega=1.0, check_every=1) as ctx:
        kappa = ctx.error_bound_factor(0, rel_tol=1e-9)
        ctx.set_options(tol=err / kappa)
        ctx.set_state(0, 0, v[: mesh.n])
        ctx.set_time_index(k0)
        ctx.step(1)
        e1 = float(np.max(np.abs(ctx.read_voltages() - v_next[: mesh.n])))
        ctx.set_options(tol=30 * err / kappa)
        ctx.set_state(0, 0, v[: mesh.n])
        ctx.set_time_index(k0)
        ctx.step(1)
        e2 = float(np.max(np.abs(ctx.read_voltages() - v_next[: mesh.n])))
    say(f"  kappa {kappa:.3f}: error {e1:.3e} at tol err/kappa, {e2:.3e} at 30x")
    assert e1 <= err
    assert e2 > e1
