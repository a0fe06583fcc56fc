"""Seeded generators for on-chip power-mesh workloads.

Mesh convention (used by every consumer):
  * ``nl`` metal layers, each an ``ny x nx`` grid; node id ``(l*ny + y)*nx + x``.
  * ``gE[l, y, x]`` is the conductance (S) of the segment between ``(l,y,x)`` and
    ``(l,y,x+1)``; ``gN[l, y, x]`` the segment between ``(l,y,x)`` and ``(l,y+1,x)``.
  * ``C[l, y, x]`` is the capacitance (F) from the node to ground.
  * A via joins node ``via_node[k]`` (layer l) to ``via_node[k] + nx*ny`` (layer
    l+1) through conductance ``via_g[k]`` in series with inductance ``via_L[k]``
    (0 means a plain resistor).
  * A pad joins node ``pad_node[k]`` to the ideal supply ``vdd`` through
    ``pad_g[k]`` in series with ``pad_L[k]`` (0 means a plain resistor).
  * A current source draws ``i(t)`` from a node to ground.  Pulses are
    symmetric triangles: zero before ``start``, rising linearly to ``peak`` at
    ``start + width/2``, back to zero at ``start + width``.

Every array is float64 (SI units) or int32.  Random draws use numpy's PCG64
through ``SeedSequence(seed).spawn(8)``; stream j draws, in this order,
0 gE, 1 gN, 2 C, 3 pulse-node choice, 4 peak, 5 start, 6 width,
7 inductances (RLC) or grid sides (uneven batch).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PS = 1e-12
PF = 1e-12
MA = 1e-3


@dataclass
class Mesh:
    nx: int
    ny: int
    nl: int
    gE: np.ndarray
    gN: np.ndarray
    C: np.ndarray
    via_node: np.ndarray
    via_g: np.ndarray
    via_L: np.ndarray
    pad_node: np.ndarray
    pad_g: np.ndarray
    pad_L: np.ndarray
    vdd: float = 1.0

    @property
    def n(self) -> int:
        return self.nl * self.ny * self.nx

    @property
    def plane(self) -> int:
        return self.ny * self.nx

    @property
    def has_inductors(self) -> bool:
        return bool(np.any(self.via_L > 0) or np.any(self.pad_L > 0))

    def node_id(self, l, y, x):
        return (np.asarray(l) * self.ny + np.asarray(y)) * self.nx + np.asarray(x)


@dataclass
class Pulses:
    """Triangular current pulses of one scenario (one pulse per listed node)."""
    node: np.ndarray   # int32, strictly increasing
    peak: np.ndarray   # A
    start: np.ndarray  # s
    width: np.ndarray  # s

    @property
    def count(self) -> int:
        return int(self.node.size)


@dataclass
class Workload:
    name: str
    meshes: List[Mesh]
    pulses: List[List[Pulses]]          # [grid][scenario]
    h: float
    steps: int
    precision: str = "fp64"             # "fp64" or "fp32+ref"
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return sum(m.n * len(p) for m, p in zip(self.meshes, self.pulses))


def _streams(seed) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(8)]


def _lattice_nodes(nx, ny, layer, step, offset=0):
    ys, xs = np.meshgrid(np.arange(offset, ny, step), np.arange(offset, nx, step),
                         indexing="ij")
    return ((layer * ny + ys) * nx + xs).ravel().astype(np.int32)


def pulse_draw(rngs, candidates: np.ndarray, fraction: Optional[float],
               peak_max=1.0 * MA, start_max=500 * PS, wmin=50 * PS, wmax=200 * PS) -> Pulses:
    """Draw one scenario of triangular pulses on ``candidates`` (all, or a fraction)."""
    if fraction is None:
        nodes = np.sort(candidates.astype(np.int32))
    else:
        k = int(round(fraction * candidates.size))
        nodes = np.sort(rngs[3].choice(candidates, size=k, replace=False).astype(np.int32))
    k = nodes.size
    peak = rngs[4].uniform(0.0, peak_max, k)
    start = rngs[5].uniform(0.0, start_max, k)
    width = rngs[6].uniform(wmin, wmax, k)
    return Pulses(nodes, peak, start, width)


def _mesh_values(rngs, nx, ny, nl, layer_g, g_jitter, c_lo, c_hi, c_layers):
    """Segment conductances ``layer_g[l] * U(jitter)`` and node caps on ``c_layers``."""
    lo, hi = g_jitter
    gE = rngs[0].uniform(lo, hi, (nl, ny, nx - 1)) * np.asarray(layer_g)[:, None, None]
    gN = rngs[1].uniform(lo, hi, (nl, ny - 1, nx)) * np.asarray(layer_g)[:, None, None]
    C = np.zeros((nl, ny, nx))
    capv = rngs[2].uniform(c_lo, c_hi, (len(c_layers), ny, nx))
    for j, l in enumerate(c_layers):
        C[l] = capv[j]
    return gE, gN, C


def _empty_i():
    return np.zeros(0, np.int32)


def _empty_f():
    return np.zeros(0)


def small_rc(nx=32, ny=32, seed=0, pad_every=8, g_range=(0.5, 2.0), c_range=(0.5 * PF, 2.0 * PF),
             pad_g=10.0, fraction=None, scenarios=1, h=10 * PS, steps=100, name=None) -> Workload:
    """Single-layer RC mesh with the 32x32 workload's value recipe at any size."""
    r = _streams(seed)
    gE, gN, C = _mesh_values(r, nx, ny, 1, [1.0], g_range, c_range[0], c_range[1], [0])
    pads = _lattice_nodes(nx, ny, 0, pad_every)
    mesh = Mesh(nx, ny, 1, gE, gN, C, _empty_i(), _empty_f(), _empty_f(),
                pads, np.full(pads.size, pad_g), np.zeros(pads.size))
    cand = np.arange(nx * ny, dtype=np.int32)
    scen = [pulse_draw(r, cand, fraction)]
    for s in range(1, scenarios):
        scen.append(pulse_draw(_streams((seed, s)), cand, fraction))
    return Workload(name or f"rc_{nx}x{ny}_s{seed}", [mesh], [scen], h, steps)


def uniform_diagonal_mesh(nx=24, ny=24, g=1.0, C=2 * PF, h=10 * PS, steps=10, vdd=1.0) -> Workload:
    """One layer of equal segments g, equal capacitance C, and a pad of k*g on every boundary
    node that misses k of its four neighbours, so every diagonal entry of the step matrix is
    C/h + 4g.  No current sources (scenarios are added by the caller)."""
    gE = np.full((1, ny, nx - 1), float(g))
    gN = np.full((1, ny - 1, nx), float(g))
    Cm = np.full((1, ny, nx), float(C))
    x, y = np.meshgrid(np.arange(nx), np.arange(ny))
    missing = (x == 0).astype(int) + (x == nx - 1) + (y == 0) + (y == ny - 1)
    node = (y * nx + x).ravel()
    k = missing.ravel()
    pads = node[k > 0].astype(np.int32)
    mesh = Mesh(nx, ny, 1, gE, gN, Cm, _empty_i(), _empty_f(), _empty_f(), pads, g * k[k > 0].astype(float),
                np.zeros(pads.size), vdd)
    empty = Pulses(_empty_i(), _empty_f(), _empty_f(), _empty_f())
    return Workload(f"uniform_diag_{nx}x{ny}", [mesh], [[empty]], h, steps)


def config0() -> Workload:
    """RC 32x32 single layer, FP64, h=10 ps, 100 steps."""
    w = small_rc(32, 32, seed=0, name="rc_32x32_fp64")
    w.precision = "fp64"
    return w


def small_multilayer(side=1024, seed=1, nl=3, layer_g=(1.0, 2.0, 4.0), via_every=4, via_g=5.0,
                     pad_every=64, pad_g=10.0, c_range=(0.1 * PF, 5.0 * PF), fraction=0.3,
                     h=10 * PS, steps=1000, via_L_range=None, pad_L_range=None, name=None) -> Workload:
    """Multi-layer mesh: decaps and pulses on the bottom layer, pads on the top one.

    With ``via_L_range``/``pad_L_range`` set, each via and pad branch is a
    resistor in series with an inductance drawn uniformly from the range.
    """
    nx = ny = side
    r = _streams(seed)
    gE, gN, C = _mesh_values(r, nx, ny, nl, list(layer_g)[:nl], (0.8, 1.2),
                             c_range[0], c_range[1], [0])
    vias = np.concatenate([_lattice_nodes(nx, ny, l, via_every) for l in range(nl - 1)]) \
        if nl > 1 else _empty_i()
    pads = _lattice_nodes(nx, ny, nl - 1, pad_every)
    via_L = np.zeros(vias.size)
    pad_L = np.zeros(pads.size)
    if via_L_range is not None:
        via_L = r[7].uniform(via_L_range[0], via_L_range[1], vias.size)
    if pad_L_range is not None:
        pad_L = r[7].uniform(pad_L_range[0], pad_L_range[1], pads.size)
    mesh = Mesh(nx, ny, nl, gE, gN, C, vias.astype(np.int32), np.full(vias.size, via_g), via_L,
                pads, np.full(pads.size, pad_g), pad_L)
    cand = np.arange(nx * ny, dtype=np.int32)
    scen = [pulse_draw(r, cand, fraction)]
    return Workload(name or f"mesh_{nl}x{side}^2_s{seed}", [mesh], [scen], h, steps)


def config1(side=1024, steps=1000) -> Workload:
    """RC 3 layers x 1024^2 (3,145,728 nodes), FP32 sweeps + FP64 refinement."""
    w = small_multilayer(side=side, seed=1, nl=3, steps=steps,
                         name=f"rc_3x{side}x{side}" + ("" if side == 1024 else "_reduced"))
    w.precision = "fp32+ref"
    return w


def small_rlc(side=512, seed=2, steps=2000, name=None) -> Workload:
    """Two-layer RLC mesh: 5 S vias and 10 S pads each in series with L ~ U[1,10] pH."""
    w = small_multilayer(side=side, seed=seed, nl=2, layer_g=(1.0, 4.0), h=1 * PS, steps=steps,
                         via_L_range=(1 * PS, 10 * PS), pad_L_range=(1 * PS, 10 * PS),
                         name=name or f"rlc_2x{side}x{side}")
    return w


def config2(side=512, steps=2000) -> Workload:
    """RLC 2 layers x 512^2, h = 1 ps, 2000 steps."""
    w = small_rlc(side=side, seed=2, steps=steps,
                  name=f"rlc_2x{side}x{side}" + ("" if side == 512 else "_reduced"))
    w.precision = "fp32+ref"
    return w


def _c3_mesh_and_pulses(seed, side):
    r = _streams(seed)
    gE, gN, C = _mesh_values(r, side, side, 1, [1.0], (0.5, 2.0), 0.5 * PF, 2.0 * PF, [0])
    pads = _lattice_nodes(side, side, 0, 8)
    mesh = Mesh(side, side, 1, gE, gN, C, _empty_i(), _empty_f(), _empty_f(),
                pads, np.full(pads.size, 10.0), np.zeros(pads.size))
    return r, mesh


def config3a(side=256, scenarios=256, steps=500) -> Workload:
    """256 current scenarios sharing one 256x256 RC mesh (32x32 workload's values)."""
    r, mesh = _c3_mesh_and_pulses(3, side)
    cand = np.arange(side * side, dtype=np.int32)
    scen = [pulse_draw(_streams((3, s)), cand, None) for s in range(scenarios)]
    return Workload(f"batch_{scenarios}scen_{side}x{side}", [mesh], [scen], 10 * PS, steps,
                    precision="fp32+ref")


def config3b(n_grids=64, sides=(64, 128, 256, 512), steps=500) -> Workload:
    """64 independent RC grids with sides drawn uniformly from {64,128,256,512}."""
    r = _streams(3)
    side_draw = r[7].choice(np.asarray(sides), size=n_grids)
    meshes, pulses = [], []
    for g, s in enumerate(side_draw):
        rg, mesh = _c3_mesh_and_pulses((3, 1000 + g), int(s))
        meshes.append(mesh)
        pulses.append([pulse_draw(rg, np.arange(int(s) ** 2, dtype=np.int32), None)])
    return Workload(f"batch_{n_grids}grids_uneven", meshes, pulses, 10 * PS, steps,
                    precision="fp32+ref", extra={"sides": side_draw.tolist()})


def config4(side=1024, steps=200) -> Workload:
    """Single-layer 1024^2 RC mesh for the adjoint: g = U[0.8,1.2] S, C ~ U[0.1,5] pF everywhere."""
    r = _streams(4)
    gE, gN, C = _mesh_values(r, side, side, 1, [1.0], (0.8, 1.2), 0.1 * PF, 5.0 * PF, [0])
    pads = _lattice_nodes(side, side, 0, 64)
    mesh = Mesh(side, side, 1, gE, gN, C, _empty_i(), _empty_f(), _empty_f(),
                pads, np.full(pads.size, 10.0), np.zeros(pads.size))
    cand = np.arange(side * side, dtype=np.int32)
    scen = [pulse_draw(r, cand, 0.3)]
    return Workload(f"adjoint_rc_{side}x{side}", [mesh], [scen], 10 * PS, steps,
                    extra={"ckpt_every": 20, "margin": 0.05})


CONFIGS = {
    "config0": config0, "config1": config1, "config2": config2,
    "config3a": config3a, "config3b": config3b, "config4": config4,
}


def random_mesh(seed, nx, ny, nl, scenarios=1, inductive=False, h=10 * PS, steps=12) -> Workload:
    """A random layered mesh for property tests: segments U[0.5,2] S, capacitance U[0.1,5] pF
    on about 70% of the nodes, vias on about 30% of the lower nodes (U[1,6] S; with
    ``inductive`` about half of them, and of the pads, in series with U[1,10] pH), pads
    U[5,10] S on about 10% of the top layer plus node 0 of every layer, and per scenario
    triangular loads on about half of the nodes (peak U[0,5] mA, start U[0,100] ps, width
    U[20,100] ps)."""
    r = np.random.default_rng(np.random.SeedSequence(seed))
    P = nx * ny
    gE = r.uniform(0.5, 2.0, (nl, ny, nx - 1))
    gN = r.uniform(0.5, 2.0, (nl, ny - 1, nx))
    C = r.uniform(0.1 * PF, 5.0 * PF, (nl, ny, nx)) * (r.random((nl, ny, nx)) < 0.7)
    vias = np.flatnonzero(r.random(P * (nl - 1)) < 0.3).astype(np.int32)
    via_g = r.uniform(1.0, 6.0, vias.size)
    via_L = r.uniform(1 * PS, 10 * PS, vias.size) * (r.random(vias.size) < 0.5) if inductive else np.zeros(vias.size)
    top = (nl - 1) * P + np.flatnonzero(r.random(P) < 0.1)
    pads = np.unique(np.concatenate([top, np.arange(nl) * P])).astype(np.int32)
    pad_g = r.uniform(5.0, 10.0, pads.size)
    pad_L = r.uniform(1 * PS, 10 * PS, pads.size) * (r.random(pads.size) < 0.5) if inductive else np.zeros(pads.size)
    mesh = Mesh(nx, ny, nl, gE, gN, C, vias, via_g, via_L, pads, pad_g, pad_L)
    scen = []
    for _ in range(scenarios):
        nodes = np.flatnonzero(r.random(nl * P) < 0.5).astype(np.int32)
        scen.append(Pulses(nodes, r.uniform(0.0, 5 * MA, nodes.size), r.uniform(0.0, 100 * PS, nodes.size),
                           r.uniform(20 * PS, 100 * PS, nodes.size)))
    return Workload(f"random_{nl}x{ny}x{nx}_s{seed}", [mesh], [scen], h, steps)


def random_direction(mesh, seed=2024):
    """A seeded direction in the (C, gE, gN) parameter space: each entry is its parameter's value
    with a random sign (for directional finite differences)."""
    r = np.random.default_rng(np.random.SeedSequence(seed))
    return tuple(r.choice([-1.0, 1.0], size=a.shape) * a for a in (mesh.C, mesh.gE, mesh.gN))
