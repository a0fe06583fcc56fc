"""Pins of the oracle's adjoint: central finite differences of its forward
transient per parameter, and the tangent-linear / adjoint identity."""
import numpy as np
import pytest

from oracle.adjoint import adjoint_branch_gradients, adjoint_gradients, forward_states, softplus_loss, \
    tangent_linear
from workloads import Pulses, small_rc, small_multilayer


def _mesh_case():
    w = small_rc(6, 5, seed=17, steps=16)
    mesh, p = w.meshes[0], w.pulses[0][0]
    # compress the pulses into the 16-step window and make the drop reach the margin
    p = Pulses(p.node, p.peak * 400, p.start * 0.2, p.width * 0.5)
    return w, mesh, p


def _J(mesh, p, h, steps, margin):
    _, V = forward_states(mesh, p, h, steps)
    return softplus_loss(V[1:], mesh.vdd, margin)


def test_adjoint_matches_central_differences():
    w, mesh, p = _mesh_case()
    h, K, margin = w.h, 16, 0.05
    J, dC, dgE, dgN = adjoint_gradients(mesh, p, h, K, margin)
    assert abs(J - _J(mesh, p, h, K, margin)) < 1e-12 * J
    rng = np.random.default_rng(0)
    checks = 0
    for arr, grad in ((mesh.C, dC), (mesh.gE, dgE), (mesh.gN, dgN)):
        flat = arr.reshape(-1)
        for j in rng.choice(flat.size, size=8, replace=False):
            base = flat[j]
            step = 1e-5 * base
            flat[j] = base + step; Jp = _J(mesh, p, h, K, margin)
            flat[j] = base - step; Jm = _J(mesh, p, h, K, margin)
            flat[j] = base
            fd = (Jp - Jm) / (2 * step)
            g = grad.reshape(-1)[j]
            assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * np.max(np.abs(grad))), (fd, g)
            checks += 1
    assert checks == 24


def test_via_and_pad_gradients_match_central_differences():
    """Two layers with vias every 2 nodes and pads every 3: dJ/dg of every via and every pad."""
    w = small_multilayer(side=6, seed=19, nl=2, via_every=2, pad_every=3, fraction=1.0, steps=14)
    mesh, p = w.meshes[0], w.pulses[0][0]
    p = Pulses(p.node, p.peak * 400, p.start * 0.2, p.width * 0.5)
    h, K, margin = w.h, 14, 0.05
    dvia, dpad = adjoint_branch_gradients(mesh, p, h, K, margin)
    assert dvia.size == mesh.via_node.size and dpad.size == mesh.pad_node.size
    for arr, grad in ((mesh.via_g, dvia), (mesh.pad_g, dpad)):
        for j in range(arr.size):
            base = arr[j]
            step = 1e-5 * base
            arr[j] = base + step; Jp = _J(mesh, p, h, K, margin)
            arr[j] = base - step; Jm = _J(mesh, p, h, K, margin)
            arr[j] = base
            fd = (Jp - Jm) / (2 * step)
            assert abs(fd - grad[j]) <= 1e-6 * max(abs(grad[j]), 1e-3 * np.max(np.abs(grad))), (fd, grad[j])
    assert np.max(np.abs(dpad)) > 0 and np.max(np.abs(dvia)) > 0


def test_tangent_linear_equals_adjoint_projection():
    w = small_multilayer(side=7, seed=3, nl=1, pad_every=3, fraction=1.0, steps=12)
    mesh, p = w.meshes[0], w.pulses[0][0]
    p = Pulses(p.node, p.peak * 300, p.start * 0.2, p.width * 0.5)
    J, dC, dgE, dgN = adjoint_gradients(mesh, p, w.h, 12, 0.05)
    rng = np.random.default_rng(5)
    d = [rng.standard_normal(a.shape) * a for a in (mesh.C, mesh.gE, mesh.gN)]
    tl = tangent_linear(mesh, p, w.h, 12, 0.05, *d)
    adj = np.sum(dC * d[0]) + np.sum(dgE * d[1]) + np.sum(dgN * d[2])
    assert abs(tl - adj) < 1e-10 * abs(adj)


def test_adjoint_rejects_inductors():
    from workloads import small_rlc
    w = small_rlc(side=4, seed=1, steps=2)
    with pytest.raises(ValueError):
        adjoint_gradients(w.meshes[0], w.pulses[0][0], w.h, 2, 0.05)
