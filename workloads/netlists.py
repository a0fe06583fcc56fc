"""Seeded general netlists (the paper's branch form, Sec. III) for the colour-ordered path.

Netlist convention (as in ``pg_validate_netlist``): trivial nodes ``0 .. n-1``, source
node ``n + j`` is an ideal supply of voltage ``source_v[j]`` with its negative terminal
grounded, ``-1`` is ground.  ``kind`` is 'R' (value = conductance, S), 'C' (F), 'L' (H)
or 'I' (a current source from ``frm`` to ground; its waveform is the matching entry of the
scenario's ``Pulses``, in branch order, and its value is that index).

``irregular_grid`` is a layered power grid whose graph is not a regular mesh: segments are
dropped at random, diagonal straps join (x, y) to (x+1, y+1) (so the graph is not bipartite),
capacitors couple neighbouring nodes, some nodes leak to ground, pads go to two supplies of
different voltage, and in the RLC variant vias carry a series R-L (through an internal node)
and some pads are pure inductors.  Node ids can be shuffled, so nothing may rely on a
geometric numbering.  ``mesh_netlist`` writes a layered ``Mesh`` as such a branch list.

Random draws use numpy's PCG64 through ``SeedSequence(seed).spawn(10)``; stream j draws, in
this order, 0 segment drops, 1 segment conductances, 2 diagonal straps, 3 capacitances,
4 coupling pairs and values, 5 leaks, 6 inductances, 7 pulse nodes, 8 pulse shapes,
9 the node shuffle.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .grids import MA, PF, PS, Mesh, Pulses

PH = 1e-12


@dataclass
class Netlist:
    n: int
    source_v: np.ndarray   # (p,)
    frm: np.ndarray        # int32
    to: np.ndarray         # int32
    kind: np.ndarray       # '<U1'
    value: np.ndarray      # float64

    @property
    def p(self) -> int:
        return int(self.source_v.size)

    @property
    def m(self) -> int:
        return int(self.frm.size)

    def source_nodes(self) -> np.ndarray:
        """Trivial node of every current source, in branch order."""
        return self.frm[self.kind == "I"].astype(np.int32)


class _Branches:
    def __init__(self):
        self.f, self.t, self.k, self.v = [], [], [], []

    def add(self, a, b, k, v):
        a = np.asarray(a, np.int64).ravel()
        b = np.broadcast_to(np.asarray(b, np.int64).ravel(), a.shape)
        v = np.broadcast_to(np.asarray(v, float).ravel(), a.shape)
        self.f.append(a); self.t.append(np.array(b)); self.k.append(np.full(a.size, k)); self.v.append(np.array(v))

    def build(self, n, source_v) -> Netlist:
        cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
        return Netlist(int(n), np.asarray(source_v, float), cat(self.f, np.int32), cat(self.t, np.int32),
                       cat(self.k, "<U1"), cat(self.v, np.float64))


def _pulses(rng_node, rng_shape, nodes, fraction, peak_max, start_max, wmin, wmax) -> Pulses:
    k = int(round(fraction * nodes.size))
    sel = np.sort(rng_node.choice(nodes, size=k, replace=False).astype(np.int32))
    peak = rng_shape.uniform(0.0, peak_max, k)
    start = rng_shape.uniform(0.0, start_max, k)
    width = rng_shape.uniform(wmin, wmax, k)
    return Pulses(sel, peak, start, width)


def _reconnect(rng, side, keepE, keepN):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    P = side * side
    ids = np.arange(P).reshape(side, side)
    for l in range(keepE.shape[0]):
        a = np.concatenate([ids[:, :-1][keepE[l]], ids[:-1, :][keepN[l]]])
        b = np.concatenate([ids[:, 1:][keepE[l]], ids[1:, :][keepN[l]]])
        ncomp, lab = connected_components(coo_matrix((np.ones(a.size), (a, b)), shape=(P, P)), directed=False)
        if ncomp == 1:
            continue
        # dropped segments as (kind, y, x), visited in a random order, Kruskal-style
        dE = np.argwhere(~keepE[l]); dN = np.argwhere(~keepN[l])
        cand = [(0, y, x) for y, x in dE] + [(1, y, x) for y, x in dN]
        parent = list(range(ncomp))

        def find(i):
            while parent[i] != i:
                parent[i] = parent[parent[i]]
                i = parent[i]
            return i
        for j in rng.permutation(len(cand)):
            k, y, x = cand[j]
            u = ids[y, x]
            v = ids[y, x + 1] if k == 0 else ids[y + 1, x]
            cu, cv = find(lab[u]), find(lab[v])
            if cu != cv:
                parent[cu] = cv
                if k == 0:
                    keepE[l, y, x] = True
                else:
                    keepN[l, y, x] = True
                ncomp -= 1
                if ncomp == 1:
                    break


def irregular_grid(side=40, nl=2, seed=11, drop=0.1, diag=0.05, coupling=0.05, leak=0.01,
                   layer_g=(1.0, 2.0, 4.0, 8.0), via_every=4, via_g=5.0, pad_every=8, pad_g=10.0,
                   supplies=(1.0, 1.05), c_range=(0.1 * PF, 5.0 * PF), rlc=False, fraction=0.3,
                   scenarios=1, shuffle=True, peak_max=1.0 * MA, start_max=300 * PS, wmin=50 * PS,
                   wmax=200 * PS):
    """Returns (netlist, [Pulses per scenario]); current sources sit on bottom-layer nodes."""
    rs = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(10)]
    P = side * side
    nmesh = nl * P
    ids = np.arange(nmesh, dtype=np.int64).reshape(nl, side, side)
    br = _Branches()
    # in-layer segments, a fraction dropped; dropped segments are then restored (in a random
    # order) wherever they join two otherwise separate parts of a layer, so every layer stays
    # connected and the DC matrix stays non-singular
    keepE = rs[0].random((nl, side, side - 1)) >= drop
    keepN = rs[0].random((nl, side - 1, side)) >= drop
    _reconnect(rs[0], side, keepE, keepN)
    lg = np.asarray(layer_g)[:nl, None, None]
    gE = rs[1].uniform(0.5, 2.0, (nl, side, side - 1)) * lg
    gN = rs[1].uniform(0.5, 2.0, (nl, side - 1, side)) * lg
    br.add(ids[:, :, :-1][keepE], ids[:, :, 1:][keepE], "R", gE[keepE])
    br.add(ids[:, :-1, :][keepN], ids[:, 1:, :][keepN], "R", gN[keepN])
    # diagonal straps
    dmask = rs[2].random((nl, side - 1, side - 1)) < diag
    gD = rs[2].uniform(0.5, 2.0, (nl, side - 1, side - 1)) * lg
    br.add(ids[:, :-1, :-1][dmask], ids[:, 1:, 1:][dmask], "R", gD[dmask])
    # capacitors to ground at every mesh node, and coupling capacitors to the east neighbour
    cap = rs[3].uniform(c_range[0], c_range[1], (nl, side, side))
    br.add(ids.ravel(), -1, "C", cap.ravel())
    cmask = rs[4].random((nl, side, side - 1)) < coupling
    cval = rs[4].uniform(0.1, 0.5, (nl, side, side - 1)) * c_range[1]
    br.add(ids[:, :, :-1][cmask], ids[:, :, 1:][cmask], "C", cval[cmask])
    # leakage resistors to ground
    lmask = rs[5].random(nmesh) < leak
    br.add(np.nonzero(lmask)[0], -1, "R", rs[5].uniform(1e-3, 1e-2, int(lmask.sum())))
    # vias between consecutive layers on a lattice; RLC: series R-L through an internal node
    n = nmesh
    ys, xs = np.meshgrid(np.arange(0, side, via_every), np.arange(0, side, via_every), indexing="ij")
    lat = (ys * side + xs).ravel()
    for l in range(nl - 1):
        lo = l * P + lat
        up = lo + P
        if rlc:
            q = np.arange(n, n + lo.size)
            n += lo.size
            br.add(lo, q, "R", via_g)
            br.add(q, up, "L", rs[6].uniform(1.0, 10.0, lo.size) * PH)
        else:
            br.add(lo, up, "R", via_g)
    # pads on the top layer, alternating between the supplies; RLC: every fourth pad is a pure
    # inductor and the others a series R-L
    ys, xs = np.meshgrid(np.arange(0, side, pad_every), np.arange(0, side, pad_every), indexing="ij")
    pads = ((nl - 1) * P + ys * side + xs).ravel()
    sup = np.arange(pads.size) % len(supplies)  # supply index per pad

    def src_code(j):  # placeholder for supply j (-2, -3, ...), replaced once n is known
        return -(2 + int(j))

    if rlc:
        for k, a in enumerate(pads):
            if k % 4 == 3:
                br.add([a], [src_code(sup[k])], "L", rs[6].uniform(1.0, 10.0) * PH)
            else:
                br.add([a], [n], "R", pad_g)
                br.add([n], [src_code(sup[k])], "L", rs[6].uniform(1.0, 10.0) * PH)
                n += 1
    else:
        br.add(pads, [src_code(j) for j in sup], "R", pad_g)
    # current sources on the bottom layer, one scenario each
    scen = [_pulses(rs[7], rs[8], np.arange(P, dtype=np.int32), fraction, peak_max, start_max, wmin, wmax)
            for _ in range(scenarios)]
    br.add(scen[0].node, -1, "I", np.arange(scen[0].count))
    net = br.build(n, supplies)
    # supply placeholders -> source node codes n + j
    for arr in (net.frm, net.to):
        m = arr <= -2
        arr[m] = n + (-arr[m] - 2)
    # every scenario uses the first scenario's source nodes (the I branches) with its own shapes
    for s in scen[1:]:
        s.node = scen[0].node.copy()
    if shuffle:
        perm = rs[9].permutation(n).astype(np.int32)  # old id -> new id
        for arr in (net.frm, net.to):
            m = (arr >= 0) & (arr < n)
            arr[m] = perm[arr[m]]
        order = None
        for s in scen:
            newn = perm[s.node]
            order = np.argsort(newn, kind="stable")
            s.node, s.peak, s.start, s.width = newn[order], s.peak[order], s.start[order], s.width[order]
        # the I branches in the order of the (sorted) pulse nodes
        ib = np.nonzero(net.kind == "I")[0]
        net.frm[ib] = scen[0].node
        net.value[ib] = np.arange(ib.size)
    return net, scen


def mesh_netlist(mesh: Mesh, pulses: Pulses = None) -> Netlist:
    """The branch list of a layered mesh: segments and vias as R (a via or pad with L > 0 as R
    then L through an internal node numbered after the mesh nodes), C to ground, pads to one
    supply, and one I branch per pulse in pulse order."""
    nx, ny, nl = mesh.nx, mesh.ny, mesh.nl
    ids = np.arange(mesh.n, dtype=np.int64).reshape(nl, ny, nx)
    br = _Branches()
    br.add(ids[:, :, :-1], ids[:, :, 1:], "R", mesh.gE)
    br.add(ids[:, :-1, :], ids[:, 1:, :], "R", mesh.gN)
    cm = mesh.C.ravel() > 0
    br.add(ids.ravel()[cm], -1, "C", mesh.C.ravel()[cm])
    n = mesh.n
    SUP = -2
    for near, far, g, L in ((mesh.via_node, mesh.via_node.astype(np.int64) + nx * ny, mesh.via_g, mesh.via_L),
                            (mesh.pad_node, np.full(mesh.pad_node.size, SUP), mesh.pad_g, mesh.pad_L)):
        near = np.asarray(near, np.int64)
        L = np.zeros(near.size) if L is None or np.asarray(L).size == 0 else np.asarray(L, float)
        plain = L <= 0
        br.add(near[plain], np.asarray(far)[plain], "R", np.asarray(g)[plain])
        q = np.nonzero(~plain)[0]
        if q.size:
            mid = np.arange(n, n + q.size)
            n += q.size
            br.add(near[q], mid, "R", np.asarray(g)[q])
            br.add(mid, np.asarray(far)[q], "L", L[q])
    if pulses is not None and pulses.count:
        br.add(pulses.node, -1, "I", np.arange(pulses.count))
    net = br.build(n, [mesh.vdd])
    for arr in (net.frm, net.to):
        arr[arr == SUP] = n
    return net


@dataclass
class NetWorkload:
    """General-netlist workload: one netlist per grid, scenarios of pulses per grid."""
    name: str
    nets: List[Netlist]
    pulses: List[List[Pulses]]
    h: float
    steps: int
    precision: str = "fp32+ref"
    note: str = ""
    dc_start: bool = False   # start from the DC operating point at t = 0 (not v = source_v[0])

    @property
    def nodes(self) -> int:
        return sum(n.n * len(p) for n, p in zip(self.nets, self.pulses))


def graph1(side=1024, steps=1000, shuffle=False) -> NetWorkload:
    """A 3-layer irregular RC grid at the scale of the 3-layer 1024 x 1024 mesh: 3,145,728 nodes,
    10 % of segments dropped, 5 % diagonal straps, 5 % coupling capacitors, 1 % leaks, 5 S vias
    every 4 nodes, 10 S pads every 64 nodes on the top layer alternating between 1.0 V and
    1.05 V, 30 % of the bottom layer pulsing; natural (geometric) node numbering, or with
    shuffle=True node ids in random order (as a netlist extracted from a layout may number
    them).  With two supply voltages v = 1.0 V is not a steady state, so the transient starts
    from the DC operating point at t = 0 (no load is on at t = 0)."""
    net, scen = irregular_grid(side=side, nl=3, seed=41, via_every=4, pad_every=64, fraction=0.3,
                               shuffle=shuffle, start_max=500 * PS)
    return NetWorkload(f"graph_irregular_3x{side}" + ("_shuffled" if shuffle else ""), [net], [scen], 10 * PS, steps,
                       note="irregular 3-layer RC netlist, colour-ordered sweeps", dc_start=True)


def graph_mesh1(side=1024, steps=1000) -> NetWorkload:
    """The 3-layer 1024 x 1024 RC mesh workload written as a branch list (two colours)."""
    from .grids import config1
    w = config1(side=side, steps=steps)
    mesh, p = w.meshes[0], w.pulses[0][0]
    return NetWorkload(f"graph_of_mesh_3x{side}", [mesh_netlist(mesh, p)], [[p]], w.h, steps,
                       note="the 3-layer mesh as a general netlist")
