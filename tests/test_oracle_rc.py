"""Pins of the RC part of the oracle against closed forms, hand-worked circuits
and invariants that follow from the paper's formulation (eqs. 1-3, Lemma 1)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import BEStepper, Circuit, GROUND, be_transient, dc_solve, mesh_to_circuit
from oracle.sources import currents_at
from workloads import Mesh, Pulses, small_rc, small_multilayer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_node(C=2e-12, g0=10.0, vdd=1.0, I=None):
    frm = [0, 0]; to = [1, GROUND]; kind = ["R", "C"]; val = [g0, C]
    if I is not None:
        frm.append(0); to.append(GROUND); kind.append("I"); val.append(0.0)
    return Circuit(1, np.array([vdd]), np.array(frm), np.array(to), np.array(kind), np.array(val, float))


def test_single_node_geometric_decay():
    """v_k - Vdd = (v0 - Vdd) r^k with r = (C/h)/(C/h + g0) (eq. 2 on one node)."""
    C, g0, h, vdd = 2e-12, 10.0, 1e-13, 1.0
    st = BEStepper(one_node(C, g0, vdd), h)
    r = (C / h) / (C / h + g0)
    v = np.array([0.3]); il = np.zeros(0)
    for k in range(1, 40):
        v, il = st.step(v, il, np.zeros(0))
        assert abs((v[0] - vdd) - (0.3 - vdd) * r ** k) < 1e-15


def test_single_node_constant_current_steady_state():
    C, g0, h, vdd, I = 1e-12, 4.0, 1e-12, 1.0, 0.02
    st = BEStepper(one_node(C, g0, vdd, I=True), h)
    vinf = vdd - I / g0
    r = (C / h) / (C / h + g0)
    v = np.array([vdd]); il = np.zeros(0)
    for k in range(1, 60):
        v, il = st.step(v, il, np.array([I]))
        assert abs((v[0] - vinf) - (vdd - vinf) * r ** k) < 1e-15
    assert abs(v[0] - vinf) < 1e-12


def test_backward_euler_first_order():
    """Error of BE against exp(-g0 t / C) at a fixed time halves when h halves."""
    C, g0, T = 1e-12, 1.0, 2e-12
    errs = []
    for K in (50, 100, 200, 400):
        st = BEStepper(one_node(C, g0, 1.0), T / K)
        v = np.array([0.0]); il = np.zeros(0)
        for _ in range(K):
            v, il = st.step(v, il, np.zeros(0))
        exact = 1.0 - np.exp(-g0 * T / C)
        errs.append(abs(v[0] - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.9 < q < 2.1 for q in ratios), ratios


def test_two_node_golden():
    d = json.load(open(os.path.join(GOLDEN, "two_node_rc.json")))
    p = d["values"]
    circ = Circuit(2, np.array([p["Vdd"]]),
                   np.array([0, 1, 0, 0, 1]), np.array([GROUND, GROUND, 2, 1, GROUND]),
                   np.array(["C", "C", "R", "R", "I"]),
                   np.array([p["C1"], p["C2"], p["g0"], p["g"], 0.0]))
    st = BEStepper(circ, p["h"])
    v = np.array(d["initial"]); il = np.zeros(0)
    for exp in d["expected"]:
        v, il = st.step(v, il, np.array([p["I"]]))
        want = np.array([float(Fraction(a, b)) for a, b in exp])
        assert np.max(np.abs(v - want)) < 1e-15


def _zero_pulses(p):
    return Pulses(p.node, np.zeros_like(p.peak), p.start, p.width)


def test_zero_current_stays_at_vdd():
    w = small_multilayer(side=24, seed=5, nl=3, via_every=4, pad_every=8, steps=30)
    mesh, pulses = w.meshes[0], _zero_pulses(w.pulses[0][0])
    circ, info = mesh_to_circuit(mesh, pulses)
    V, _ = be_transient(circ, info, pulses, w.h, 30)
    assert np.max(np.abs(V - mesh.vdd)) < 1e-13


def _drop(mesh, pulses, h, steps):
    circ, info = mesh_to_circuit(mesh, pulses)
    V, _ = be_transient(circ, info, pulses, h, steps)
    return mesh.vdd - V


def _subset(p, mask):
    return Pulses(p.node[mask], p.peak[mask], p.start[mask], p.width[mask])


def test_superposition_and_homogeneity():
    w = small_rc(14, 11, seed=7, steps=40)
    mesh, p = w.meshes[0], w.pulses[0][0]
    rng = np.random.default_rng(0)
    mask = rng.random(p.count) < 0.5
    dA = _drop(mesh, _subset(p, mask), w.h, 40)
    dB = _drop(mesh, _subset(p, ~mask), w.h, 40)
    dAB = _drop(mesh, p, w.h, 40)
    assert np.max(np.abs(dAB - dA - dB)) < 1e-13
    scaled = Pulses(p.node, 2.5 * p.peak, p.start, p.width)
    assert np.max(np.abs(_drop(mesh, scaled, w.h, 40) - 2.5 * dAB)) < 1e-13


@pytest.mark.parametrize("maker", [lambda: small_rc(9, 7, seed=3),
                                   lambda: small_multilayer(side=10, seed=4, nl=3, via_every=3, pad_every=5)])
def test_system_matrix_spd_lemma1(maker):
    """Lemma 1: M symmetric, weakly diagonally dominant with a strictly dominant row, PD."""
    w = maker()
    circ, _ = mesh_to_circuit(w.meshes[0], w.pulses[0][0])
    M = circ.system_matrix(w.h).toarray()
    assert np.array_equal(M, M.T)
    off = np.sum(np.abs(M), axis=1) - np.abs(np.diag(M))
    assert np.all(np.diag(M) >= off - 1e-12)
    assert np.any(np.diag(M) > off + 1e-3)
    np.linalg.cholesky(M)
    assert np.linalg.eigvalsh(M).min() > 0


def _uniform_mesh(nx, ny, nl, g, gv, C, g0):
    n = nl * nx * ny
    vias = np.arange((nl - 1) * nx * ny, dtype=np.int32)
    return Mesh(nx, ny, nl, np.full((nl, ny, nx - 1), g), np.full((nl, ny - 1, nx), g),
                np.full((nl, ny, nx), C), vias, np.full(vias.size, gv), np.zeros(vias.size),
                np.arange(n, dtype=np.int32), np.full(n, g0), np.zeros(n), vdd=1.0)


@pytest.mark.parametrize("nl", [1, 2, 3])
def test_uniform_mesh_matches_dct_diagonalisation(nl):
    """On a uniform mesh with a pad on every node, M = (C/h + G0) I + g (T_x + T_y) + g_v T_z
    where T is the path-graph Laplacian; the orthonormal DCT-II diagonalises every T with
    eigenvalues 2 - 2 cos(pi k / N).  One BE step solved that way must equal the oracle's."""
    nx, ny, g, gv, C, g0, h = 13, 9, 1.3, 4.0, 0.7e-12, 0.25, 1e-12
    mesh = _uniform_mesh(nx, ny, nl, g, gv, C, g0)
    rng = np.random.default_rng(11)
    n = mesh.n
    peak = rng.uniform(0, 1e-3, n)
    pulses = Pulses(np.arange(n, dtype=np.int32), peak, np.zeros(n), np.full(n, 2 * h))
    circ, info = mesh_to_circuit(mesh, pulses)
    V, _ = be_transient(circ, info, pulses, h, 1)
    I1 = currents_at(pulses, h)
    b = (C / h) * 1.0 + g0 * 1.0 - I1
    lam = lambda N: 2.0 - 2.0 * np.cos(np.pi * np.arange(N) / N)
    eig = (C / h + g0) + g * (lam(nx)[None, None, :] + lam(ny)[None, :, None]) \
        + gv * lam(nl)[:, None, None]
    B = sfft.dctn(b.reshape(nl, ny, nx), type=2, norm="ortho")
    v_dct = sfft.idctn(B / eig, type=2, norm="ortho").ravel()
    assert np.max(np.abs(V[0] - v_dct)) < 1e-13


def test_charge_balance_every_step():
    """KCL summed over all nodes: sum C/h (v_k+1 - v_k) + sum_pads g0 (v_p - Vdd) + sum I = 0."""
    w = small_multilayer(side=16, seed=9, nl=2, via_every=4, pad_every=8, steps=60)
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    V, _ = be_transient(circ, info, p, w.h, 60)
    Vall = np.vstack([np.full(mesh.n, mesh.vdd), V])
    C = mesh.C.ravel()
    for k in range(1, 61):
        I = currents_at(p, k * w.h).sum()
        q = np.sum(C / w.h * (Vall[k] - Vall[k - 1]))
        pad = np.sum(mesh.pad_g * (Vall[k][mesh.pad_node] - mesh.vdd))
        assert abs(q + pad + I) < 1e-12 * max(1.0, I) + 1e-15


def test_maximum_principle_and_monotone_drop():
    w = small_rc(12, 12, seed=13, steps=50)
    mesh, p = w.meshes[0], w.pulses[0][0]
    d1 = _drop(mesh, p, w.h, 50)
    d2 = _drop(mesh, Pulses(p.node, p.peak * 1.7 + 1e-5, p.start, p.width), w.h, 50)
    assert np.all(d1 >= -1e-15)
    assert np.all(d2 - d1 >= -1e-15)
    assert d1.max() > 1e-4


def test_reciprocity():
    """M^-1 symmetric: a unit source at a seen at b equals a unit source at b seen at a."""
    w = small_multilayer(side=8, seed=2, nl=2, via_every=2, pad_every=4)
    mesh = w.meshes[0]
    a, b = 5, mesh.n - 3
    resp = []
    for src, obs in ((a, b), (b, a)):
        p = Pulses(np.array([src], np.int32), np.array([1.0]), np.array([0.0]), np.array([2 * w.h]))
        resp.append(mesh.vdd - _drop_free(mesh, p, w.h)[obs])
    assert abs(resp[0] - resp[1]) < 1e-12 * abs(resp[0])


def _drop_free(mesh, p, h):
    circ, info = mesh_to_circuit(mesh, p)
    V, _ = be_transient(circ, info, p, h, 1)
    return V[0]


def test_long_transient_reaches_dc():
    """With constant sources the BE transient converges to the DC point of eq. 3 (A = G)."""
    w = small_multilayer(side=10, seed=21, nl=2, via_every=2, pad_every=5, c_range=(1e-13, 1e-12))
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    I = np.random.default_rng(1).uniform(0, 1e-3, p.count)
    st = BEStepper(circ, 1e-10)
    v = np.full(circ.n, mesh.vdd); il = np.zeros(0)
    for _ in range(3000):
        v, il = st.step(v, il, I)
    vdc, _ = dc_solve(circ, I)
    assert np.max(np.abs(v - vdc)) < 1e-12
    assert np.max(mesh.vdd - vdc) > 1e-5


def test_dense_and_sparse_solvers_agree():
    w = small_rc(30, 20, seed=1, steps=12)
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    Vd, _ = be_transient(circ, info, p, w.h, 12, dense_max=10**6)
    Vs, _ = be_transient(circ, info, p, w.h, 12, dense_max=0)
    assert np.max(np.abs(Vd - Vs)) < 1e-13


def test_incidence_matches_definition():
    """Eqs. 4-5 by brute force on a small mixed circuit."""
    circ = Circuit(3, np.array([1.0, 0.5]),
                   np.array([0, 1, 2, 3, 0, GROUND]), np.array([1, 2, 4, 2, GROUND, 1]),
                   np.array(["R", "R", "R", "L", "C", "I"]), np.array([1.0, 2.0, 3.0, 1e-9, 1e-12, 0.0]))
    A, As = circ.incidence()
    A = A.toarray(); As = As.toarray()
    for e in range(circ.m):
        for j in range(3):
            want = (1 if circ.frm[e] == j else 0) - (1 if circ.to[e] == j else 0)
            assert A[e, j] == want
        for j in range(2):
            want = (1 if circ.frm[e] == 3 + j else 0) - (1 if circ.to[e] == 3 + j else 0)
            assert As[e, j] == want


def test_scaled_residual_of_exact_step_is_roundoff_and_detects_error():
    """The assembled-system residual (no factorisation) vanishes on the direct solution and
    equals |delta| * M_ii / M_ii = |delta| for a perturbation of one node by delta."""
    from oracle import BESystem, scaled_residual
    w = small_multilayer(side=12, seed=8, nl=3, via_every=4, pad_every=6, steps=3)
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    st = BEStepper(circ, w.h)
    v0 = np.full(circ.n, mesh.vdd)
    I1 = currents_at(p, w.h)
    v1, _ = st.step(v0, np.zeros(0), I1)
    sysm = BESystem(circ, w.h)
    assert scaled_residual(sysm, v0, np.zeros(0), v1, I1) < 1e-14
    v1b = v1.copy()
    v1b[7] += 1e-6
    assert abs(scaled_residual(sysm, v0, np.zeros(0), v1b, I1) - 1e-6) < 1e-12
