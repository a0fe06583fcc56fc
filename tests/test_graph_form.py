"""General netlists on the CPU: the colouring and slot layout of the colour-ordered path
(host logic of the C ABI, no device), the generator's mesh branch list, and pins of the
oracle on circuits only a general netlist can hold (coupling capacitors, two supply voltages,
pure inductors)."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from oracle import BEStepper, Circuit, GROUND, be_transient, dc_solve, mesh_to_circuit
from oracle.sources import currents_at
from workloads import Pulses, irregular_grid, mesh_netlist, small_multilayer, small_rlc


def _pattern_edges(net):
    tri = (net.frm >= 0) & (net.frm < net.n) & (net.to >= 0) & (net.to < net.n) & (net.kind != "I")
    return net.frm[tri], net.to[tri]


@pytest.mark.parametrize("rlc", [False, True])
def test_coloring_is_proper_and_slots_follow_colours(rlc):
    net, _ = irregular_grid(side=24, nl=3, seed=5, rlc=rlc)
    color, slot, nc, ns = pg.netlist_coloring(net.n, net.p, net.source_v, net.frm, net.to, net.kind, net.value)
    a, b = _pattern_edges(net)
    assert np.all(color[a] != color[b])
    assert nc >= 3  # the diagonal straps close odd cycles
    assert np.array_equal(np.sort(np.unique(color)), np.arange(nc))
    # slots: a bijection into [0, n_slots), colours in order, each colour's block contiguous and
    # padded to whole 64-slot slices
    assert len(np.unique(slot)) == net.n and slot.min() >= 0 and slot.max() < ns and ns % 64 == 0
    start = 0
    for c in range(nc):
        nodes = np.nonzero(color == c)[0]
        assert np.array_equal(np.sort(slot[nodes]), start + np.arange(nodes.size))
        start += -(-nodes.size // 64) * 64
    assert start == ns


def _cuthill_mckee(n, a, b):
    """Breadth first from a pseudo-peripheral node of each connected part (parts by smallest node),
    unvisited neighbours by increasing degree, ties by node."""
    nbrs = [set() for _ in range(n)]
    for x, y in zip(a.tolist(), b.tolist()):
        nbrs[x].add(y)
        nbrs[y].add(x)
    deg = [len(s) for s in nbrs]
    key = lambda u: (deg[u], u)
    placed, order = [False] * n, []
    for s0 in range(n):
        if placed[s0]:
            continue
        root, depth = s0, -1
        for _ in range(8):
            lev = {root: 0}
            q = [root]
            for u in q:
                for w in sorted(nbrs[u]):
                    if w not in lev:
                        lev[w] = lev[u] + 1
                        q.append(w)
            d = lev[q[-1]]
            if d <= depth:
                break
            depth = d
            root = min((u for u in q if lev[u] == d), key=key)
        placed[root] = True
        q = [root]
        for u in q:
            order.append(u)
            new = sorted((w for w in nbrs[u] if not placed[w]), key=key)
            for w in new:
                placed[w] = True
            q.extend(new)
    return order


@pytest.mark.parametrize("seed", [5, 11])
def test_slots_follow_cuthill_mckee_order_inside_each_colour(seed):
    net, _ = irregular_grid(side=20, nl=3, seed=seed)
    color, slot, nc, ns = pg.netlist_coloring(net.n, net.p, net.source_v, net.frm, net.to, net.kind, net.value)
    a, b = _pattern_edges(net)
    order = _cuthill_mckee(net.n, a, b)
    assert sorted(order) == list(range(net.n))
    for c in range(nc):
        in_c = [u for u in order if color[u] == c]
        assert np.all(np.diff(slot[in_c]) == 1)
    # neighbours lie close in this order: the widest gap along a branch is a small fraction of n
    rank = np.empty(net.n, dtype=np.int64)
    rank[order] = np.arange(net.n)
    assert np.max(np.abs(rank[a] - rank[b])) < net.n // 4


def test_mesh_branch_list_is_two_coloured_checkerboard():
    w = small_multilayer(side=20, seed=3, nl=3, pad_every=8, steps=2)
    mesh = w.meshes[0]
    net = mesh_netlist(mesh, w.pulses[0][0])
    color, _, nc, _ = pg.netlist_coloring(net.n, net.p, net.source_v, net.frm, net.to, net.kind, net.value)
    assert nc == 2
    l, y, x = np.unravel_index(np.arange(mesh.n), (mesh.nl, mesh.ny, mesh.nx))
    par = (l + y + x) % 2
    # breadth-first parity: one colour per checkerboard class (up to a swap)
    assert np.all(color[: mesh.n] == par) or np.all(color[: mesh.n] == 1 - par)


def test_odd_cycle_takes_three_colours():
    # a resistor triangle with a capacitor at every node and one pad
    net_f = np.array([0, 1, 2, 0, 1, 2, 0]); net_t = np.array([1, 2, 0, -1, -1, -1, 3])
    kind = np.array(list("RRRCCCR")); val = np.array([1.0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 2.0])
    color, slot, nc, ns = pg.netlist_coloring(3, 1, [1.0], net_f, net_t, kind, val)
    assert nc == 3 and sorted(color.tolist()) == [0, 1, 2] and ns == 3 * 64


def test_coloring_reports_invalid_netlists():
    with pytest.raises(pg.PgError) as e:
        pg.netlist_coloring(2, 1, [1.0], [0, 1], [1, -1], ["R", "X"], [1.0, 1.0])
    assert e.value.status == -1
    with pytest.raises(pg.PgError) as e:  # node 1 reaches nothing but ground
        pg.netlist_coloring(2, 1, [1.0], [0, 1], [2, -1], ["R", "C"], [1.0, 1e-12])
    assert e.value.status == -2


def test_mesh_branch_list_maps_back_to_the_mesh():
    """The generator's branch list of a mesh is the mesh (series R-L vias and pads included)."""
    w = small_rlc(side=12, seed=9, steps=2)
    mesh = w.meshes[0]
    net = mesh_netlist(mesh)
    back = pg.netlist_to_mesh(net.n, net.p, net.source_v, net.frm, net.to, net.kind, net.value,
                              (mesh.nx, mesh.ny, mesh.nl))
    assert np.array_equal(back.gE, mesh.gE) and np.array_equal(back.gN, mesh.gN) and np.array_equal(back.C, mesh.C)
    o = np.argsort(mesh.via_node, kind="stable")
    assert np.array_equal(back.via_node, mesh.via_node[o]) and np.allclose(back.via_L, mesh.via_L[o], rtol=0, atol=0)
    o = np.argsort(mesh.pad_node, kind="stable")
    assert np.array_equal(back.pad_node, mesh.pad_node[o]) and np.array_equal(back.pad_g, mesh.pad_g[o])


# ---- oracle pins on general-netlist circuits ------------------------------------------------

def _coupled_pair(C0, Cc, g, vdd):
    """Nodes 0 and 1: C0 to ground and g to the supply (code 2) each, Cc between them, and a
    current source at each node (branches 5 and 6)."""
    frm = np.array([0, 1, 0, 1, 0, 0, 1]); to = np.array([GROUND, GROUND, 2, 2, 1, GROUND, GROUND])
    kind = np.array(list("CCRRCII")); val = np.array([C0, C0, g, g, Cc, 0.0, 1.0])
    return Circuit(2, np.array([vdd]), frm, to, kind, val)


def test_coupling_capacitor_modes_follow_scalar_recurrences():
    """Equal and opposite loads on a symmetric coupled pair split into a common mode that sees
    C0 and a differential mode that sees C0 + 2 Cc; under backward Euler each mode is the scalar
    recurrence x' = (c/h x - f) / (c/h + g)."""
    C0, Cc, g, vdd, h = 2e-12, 0.7e-12, 3.0, 1.0, 1e-12
    circ = _coupled_pair(C0, Cc, g, vdd)
    pul = Pulses(np.array([0, 1], np.int32), np.array([2e-3, -1e-3]), np.array([5e-12, 5e-12]),
                 np.array([40e-12, 40e-12]))
    steps = 80
    V, _ = be_transient(circ, None, pul, h, steps, v0=np.full(2, vdd), il0=np.zeros(0))
    s = d = dmax = 0.0  # common mode (v0 + v1)/2 - vdd and differential v0 - v1
    for k in range(1, steps + 1):
        I = currents_at(pul, k * h)
        s = (C0 / h * s - 0.5 * (I[0] + I[1])) / (C0 / h + g)
        d = ((C0 + 2 * Cc) / h * d - (I[0] - I[1])) / ((C0 + 2 * Cc) / h + g)
        v = V[k - 1]
        assert abs(0.5 * (v[0] + v[1]) - vdd - s) < 1e-14
        assert abs((v[0] - v[1]) - d) < 1e-14
        dmax = max(dmax, abs(d))
    assert dmax > 1e-4  # the differential mode was driven


def test_two_supplies_dc_is_the_resistive_divider():
    """Node 0 joined to supplies of 1.0 V and 1.2 V through g1 and g2 (and a capacitor): the DC
    point is the weighted mean, and the transient from any start relaxes to it."""
    g1, g2, v1, v2 = 2.0, 6.0, 1.0, 1.2
    circ = Circuit(1, np.array([v1, v2]), np.array([0, 0, 0]), np.array([1, 2, GROUND]), np.array(list("RRC")),
                   np.array([g1, g2, 1e-12]))
    v, _ = dc_solve(circ, np.zeros(0))
    assert abs(v[0] - (g1 * v1 + g2 * v2) / (g1 + g2)) < 1e-15
    V, _ = be_transient(circ, None, None, 1e-12, 200, v0=np.array([v1]), il0=np.zeros(0))
    assert abs(V[-1, 0] - v[0]) < 1e-12


def test_pure_inductor_pad_holds_the_node_at_the_supply_at_dc():
    """A node fed only through a pure L pad (plus a load and a capacitor): BE drives it to the
    supply with the inductor carrying the load, and each step obeys C(v'-v)/h + i' + I = 0,
    L(i'-i)/h = v' - Vdd (a 2x2 solve written out)."""
    C, L, vdd, h, I = 1e-12, 2e-12, 1.0, 1e-12, 1e-3
    circ = Circuit(1, np.array([vdd]), np.array([0, 0, 0]), np.array([1, GROUND, GROUND]), np.array(list("LCI")),
                   np.array([L, C, 0.0]))
    st = BEStepper(circ, h)
    v, il = np.array([vdd]), np.zeros(1)
    x, y = vdd, 0.0
    det = (C / h) * (L / h) + 1.0
    for _ in range(3000):
        b1 = C / h * x - I
        b2 = L / h * y - vdd
        # [[C/h, 1], [-1, L/h]] [v', i'] = [b1, b2]
        x, y = (b1 * (L / h) - b2) / det, ((C / h) * b2 + b1) / det
        v, il = st.step(v, il, np.array([I]))
        assert abs(v[0] - x) < 1e-12 and abs(il[0] - y) < 1e-12
    assert abs(v[0] - vdd) < 1e-5 and abs(il[0] + I) < 1e-5
