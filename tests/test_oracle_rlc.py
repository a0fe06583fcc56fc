"""Pins of the RLC part of the oracle (eqs. 9-11, Lemma 1 with inductors)."""
import json
import os
from fractions import Fraction

import numpy as np

from oracle import BEStepper, Circuit, GROUND, be_transient, dc_solve, mesh_to_circuit, \
    three_level_transient
from oracle.sources import currents_at
from workloads import Pulses, small_rlc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tank(C, R, L, vdd):
    """Node 0 with C to ground and a current source; R from node 0 to internal node 1;
    L from node 1 to the supply (code 2)."""
    return Circuit(2, np.array([vdd]), np.array([0, 0, 1, 0]), np.array([GROUND, 1, 2, GROUND]),
                   np.array(["C", "R", "L", "I"]), np.array([C, 1.0 / R, L, 0.0]))


def test_rl_tank_golden():
    d = json.load(open(os.path.join(GOLDEN, "rl_tank.json")))
    p = d["values"]
    st = BEStepper(tank(p["C"], p["R"], p["L"], p["Vdd"]), p["h"])
    # internal node starts at the value that makes the resistor carry the initial current
    v = np.array([d["initial"]["v"], d["initial"]["v"] - p["R"] * d["initial"]["i"]])
    il = np.array([d["initial"]["i"]])
    for ev, ei in zip(d["expected_v"], d["expected_i"]):
        v, il = st.step(v, il, np.array([p["I"]]))
        assert abs(v[0] - float(Fraction(*ev))) < 1e-15
        assert abs(il[0] - float(Fraction(*ei))) < 1e-15


def test_rl_tank_matches_cramer_recurrence():
    """C (v'-v)/h + i' + I = 0 and L (i'-i)/h = v' - Vdd - R i', solved by Cramer's rule."""
    C, R, L, vdd, h, I = 1.5e-12, 0.1, 3e-12, 1.0, 1e-12, 2e-3
    st = BEStepper(tank(C, R, L, vdd), h)
    v = np.array([vdd, vdd]); il = np.zeros(1)
    x = np.array([vdd, 0.0])
    a11, a12 = C / h, 1.0
    a21, a22 = -1.0, L / h + R
    det = a11 * a22 - a12 * a21
    for _ in range(200):
        b1 = C / h * x[0] - I
        b2 = L / h * x[1] - vdd
        x = np.array([(b1 * a22 - a12 * b2) / det, (a11 * b2 - a21 * b1) / det])
        v, il = st.step(v, il, np.array([I]))
        assert abs(v[0] - x[0]) < 1e-13 and abs(il[0] - x[1]) < 1e-13 * max(1, abs(x[1]))
    # the tank settles at Vdd - R I with the inductor carrying -I
    assert abs(x[0] - (vdd - R * I)) < 1e-6


def test_rlc_mesh_system_matrix_spd():
    w = small_rlc(side=8, seed=3, steps=5)
    circ, info = mesh_to_circuit(w.meshes[0], w.pulses[0][0])
    M = circ.system_matrix(w.h).toarray()
    assert np.array_equal(M, M.T)
    off = np.sum(np.abs(M), axis=1) - np.abs(np.diag(M))
    assert np.all(np.diag(M) >= off - 1e-9)
    assert np.linalg.eigvalsh(M).min() > 0
    assert circ.n == w.meshes[0].n + w.meshes[0].via_node.size + w.meshes[0].pad_node.size


def test_three_level_recurrence_matches_two_level():
    """Eq. 11 seeded with the BE v(0), v(h) reproduces the eq. 10 trajectory."""
    w = small_rlc(side=8, seed=4, steps=40)
    mesh, p = w.meshes[0], w.pulses[0][0]
    p = Pulses(p.node, p.peak * 50, p.start * 0.02, p.width * 0.1)  # activity inside 40 ps
    circ, info = mesh_to_circuit(mesh, p)
    V, IL = be_transient(circ, info, p, w.h, 40)
    v0 = np.full(circ.n, mesh.vdd)
    V3 = three_level_transient(circ, p, w.h, 40, v0, V[0])
    scale = np.max(np.abs(V - mesh.vdd))
    assert scale > 1e-4
    assert np.max(np.abs(V3 - V[1:])) < 1e-9 * max(1.0, scale)


def test_companion_form_matches_internal_node_form():
    """Eliminating each series R-L internal node gives the companion model
    g_eq = h/(L + hR), alpha = L/(L + hR); solved densely here from scratch."""
    w = small_rlc(side=6, seed=8, steps=30)
    mesh, p = w.meshes[0], w.pulses[0][0]
    p = Pulses(p.node, p.peak * 20, p.start * 0.03, p.width * 0.1)
    circ, info = mesh_to_circuit(mesh, p)
    V, IL = be_transient(circ, info, p, w.h, 30)
    h, n, vdd, P = w.h, mesh.n, mesh.vdd, mesh.ny * mesh.nx
    M = np.zeros((n, n))
    ids = np.arange(n).reshape(mesh.nl, mesh.ny, mesh.nx)
    for a, b, g in ((ids[:, :, :-1], ids[:, :, 1:], mesh.gE), (ids[:, :-1, :], ids[:, 1:, :], mesh.gN)):
        for ai, bi, gi in zip(a.ravel(), b.ravel(), g.ravel()):
            M[ai, ai] += gi; M[bi, bi] += gi; M[ai, bi] -= gi; M[bi, ai] -= gi
    M += np.diag(mesh.C.ravel() / h)
    geq_v = h / (mesh.via_L + h / mesh.via_g); al_v = mesh.via_L / (mesh.via_L + h / mesh.via_g)
    geq_p = h / (mesh.pad_L + h / mesh.pad_g); al_p = mesh.pad_L / (mesh.pad_L + h / mesh.pad_g)
    for k, lo in enumerate(mesh.via_node):
        hi = lo + P
        M[lo, lo] += geq_v[k]; M[hi, hi] += geq_v[k]; M[lo, hi] -= geq_v[k]; M[hi, lo] -= geq_v[k]
    for k, a in enumerate(mesh.pad_node):
        M[a, a] += geq_p[k]
    v = np.full(n, vdd); iv = np.zeros(mesh.via_node.size); ip = np.zeros(mesh.pad_node.size)
    nv = mesh.via_node.size
    for k in range(1, 31):
        b = mesh.C.ravel() / h * v
        np.subtract.at(b, p.node, currents_at(p, k * h))
        np.subtract.at(b, mesh.via_node, al_v * iv)
        np.add.at(b, mesh.via_node + P, al_v * iv)
        np.subtract.at(b, mesh.pad_node, al_p * ip)
        np.add.at(b, mesh.pad_node, geq_p * vdd)
        v = np.linalg.solve(M, b)
        iv = al_v * iv + geq_v * (v[mesh.via_node] - v[mesh.via_node + P])
        ip = al_p * ip + geq_p * (v[mesh.pad_node] - vdd)
        assert np.max(np.abs(v - V[k - 1][:n])) < 1e-12
        assert np.max(np.abs(iv - IL[k - 1][:nv])) < 1e-12
        assert np.max(np.abs(ip - IL[k - 1][nv:])) < 1e-12


def test_source_free_energy_non_increasing():
    """Passivity of BE: 1/2 sum C (v - Vdd)^2 + 1/2 sum L i^2 never grows without sources."""
    w = small_rlc(side=8, seed=6, steps=80)
    mesh = w.meshes[0]
    circ, info = mesh_to_circuit(mesh, None)
    rng = np.random.default_rng(3)
    v = mesh.vdd + rng.uniform(-0.05, 0.05, circ.n)
    il = rng.uniform(-1e-2, 1e-2, int(np.sum(circ.kind == "L")))
    st = BEStepper(circ, w.h)
    Cn = circ.matrices()["C"].diagonal()
    Lv = circ.matrices()["Lvals"]
    E = lambda v, il: 0.5 * np.sum(Cn * (v - mesh.vdd) ** 2) + 0.5 * np.sum(Lv * il ** 2)
    e0 = e_prev = E(v, il)
    for _ in range(80):
        v, il = st.step(v, il, np.zeros(0))
        e = E(v, il)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e
    assert e_prev < 0.5 * e0


def test_rlc_long_transient_reaches_dc():
    w = small_rlc(side=6, seed=10, steps=5)
    mesh, p = w.meshes[0], w.pulses[0][0]
    circ, info = mesh_to_circuit(mesh, p)
    I = np.random.default_rng(2).uniform(0, 1e-3, p.count)
    st = BEStepper(circ, 2e-11)
    v = np.full(circ.n, mesh.vdd); il = np.zeros(int(np.sum(circ.kind == "L")))
    for _ in range(4000):
        v, il = st.step(v, il, I)
    vdc, ildc = dc_solve(circ, I)
    assert np.max(np.abs(v - vdc)) < 1e-10
    assert np.max(np.abs(il - ildc)) < 1e-10
    assert abs(np.sum(ildc[-mesh.pad_node.size:]) + I.sum()) < 1e-12
