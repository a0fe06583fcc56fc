"""Write the sampled oracle trajectories under ``tests/golden/`` (FP64 CPU oracle only).

Usage:  python tests/golden/make_golden.py <name> [...]
        names: config0, config1, config2, config3a, config3b, config4, config4_adjoint

Each file holds, for every backward-Euler step k = 1..K of one seeded workload, the oracle's
voltages at a fixed, seeded set of sampled nodes (stored as the drop below the supply,
``vdd - v``, in float32: at drops of a few tens of millivolts that keeps ~3e-9 V), and over all
nodes the largest drop, the node that has it and the sum of the drops.  Tests and ``bench.py``
compare the HIP path's states with these values; nothing in them comes from the HIP path.

The steps are eq. 2 (RC) or eq. 10 (RLC, companion form) solved directly by the oracle's
``BEStepper``; only ``oracle`` and the seeded input generators of ``workloads`` are used.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import BEStepper, mesh_to_circuit  # noqa: E402
from oracle.sources import currents_at  # noqa: E402
from oracle.transient import initial_state  # noqa: E402
from workloads import config0, config1, config2, config3a, config3b, config4, random_direction  # noqa: E402

SAMPLE_SEED = 71660


def sample_nodes(mesh, n_random=256):
    """The bottom-layer nodes farthest from the pad lattice (one per 64x64 pad cell, or per
    8x8 cell on small meshes), then ``n_random`` distinct seeded nodes over every layer."""
    cell = 64 if mesh.nx >= 256 else 8
    ys, xs = np.meshgrid(np.arange(cell // 2, mesh.ny, cell), np.arange(cell // 2, mesh.nx, cell),
                         indexing="ij")
    far = (ys * mesh.nx + xs).ravel()[:256]
    rng = np.random.default_rng(np.random.SeedSequence(SAMPLE_SEED))
    rest = np.setdiff1d(np.arange(mesh.n), far)
    rnd = rng.choice(rest, size=min(n_random, rest.size), replace=False)
    return np.concatenate([far, np.sort(rnd)]).astype(np.int64)


def trajectory(mesh, pulses, h, steps, nodes, log_every=50, tag=""):
    """Run the oracle over ``steps`` steps; return the per-step arrays stored in the file."""
    circ, info = mesh_to_circuit(mesh, pulses)
    n_mesh = info["n_mesh"]
    t0 = time.time()
    st = BEStepper(circ, h)
    print(f"{tag}: factored n={circ.n} in {time.time() - t0:.1f} s", flush=True)
    v, il = initial_state(circ, info, mesh.vdd)
    drops = np.empty((steps, nodes.size), np.float32)
    max_drop = np.empty(steps)
    argmax = np.empty(steps, np.int64)
    sum_drop = np.empty(steps)
    il_out = []
    t1 = time.time()
    for k in range(1, steps + 1):
        v, il = st.step(v, il, currents_at(pulses, k * h))
        d = mesh.vdd - v[:n_mesh]
        drops[k - 1] = d[nodes]
        j = int(np.argmax(d))
        argmax[k - 1] = j
        max_drop[k - 1] = d[j]
        sum_drop[k - 1] = float(np.sum(d))
        if il.size:
            il_out.append(il.copy())
        if k % log_every == 0 or k == steps:
            print(f"{tag}: step {k}/{steps}, {(time.time() - t1) / k:.3f} s/step, "
                  f"max drop {max_drop[k - 1]:.4e} V", flush=True)
    out = dict(nodes=nodes, drops=drops, max_drop=max_drop, argmax=argmax, sum_drop=sum_drop,
               h=np.float64(h), vdd=np.float64(mesh.vdd), steps=np.int64(steps))
    if il_out:
        out["il"] = np.array(il_out)
    return out


def make_config1():
    w = config1()
    mesh, p = w.meshes[0], w.pulses[0][0]
    out = trajectory(mesh, p, w.h, w.steps, sample_nodes(mesh), tag=w.name)
    np.savez_compressed(os.path.join(HERE, "config1_rc_3x1024x1024_samples.npz"),
                        workload=np.array(w.name), **out)


def make_config3a(scenarios=(0, 1, 2, 3, 85, 170, 254, 255)):
    """Sampled scenarios of the 256-scenario batch (the batch's first, last and spread ones)."""
    w = config3a()
    mesh = w.meshes[0]
    nodes = sample_nodes(mesh, n_random=192)
    res = {}
    for s in scenarios:
        o = trajectory(mesh, w.pulses[0][s], w.h, w.steps, nodes, log_every=100, tag=f"{w.name}[{s}]")
        for key in ("drops", "max_drop", "argmax", "sum_drop"):
            res.setdefault(key, []).append(o[key])
    np.savez_compressed(os.path.join(HERE, "config3a_batch_256scen_256x256_samples.npz"),
                        workload=np.array(w.name), scenarios=np.array(scenarios, np.int64),
                        nodes=nodes, h=np.float64(w.h), vdd=np.float64(mesh.vdd),
                        steps=np.int64(w.steps), **{k: np.array(v) for k, v in res.items()})


def make_config2():
    w = config2()
    mesh, p = w.meshes[0], w.pulses[0][0]
    out = trajectory(mesh, p, w.h, w.steps, sample_nodes(mesh), log_every=100, tag=w.name)
    il = out.pop("il")
    # branch currents (vias then pads in the mesh's order) of a seeded sample of 448 vias and
    # every pad, every 10th step
    rng = np.random.default_rng(np.random.SeedSequence(SAMPLE_SEED + 2))
    nv = mesh.via_node.size
    br = np.concatenate([np.sort(rng.choice(nv, size=min(448, nv), replace=False)), nv + np.arange(mesh.pad_node.size)])
    out["il_branches"] = br.astype(np.int64)
    out["il_every10"] = il[9::10][:, br].astype(np.float64)
    np.savez_compressed(os.path.join(HERE, "config2_rlc_2x512x512_samples.npz"),
                        workload=np.array(w.name), **out)


def make_config0():
    w = config0()
    mesh, p = w.meshes[0], w.pulses[0][0]
    out = trajectory(mesh, p, w.h, w.steps, np.arange(mesh.n, dtype=np.int64), log_every=50, tag=w.name)
    np.savez_compressed(os.path.join(HERE, "config0_rc_32x32_all_nodes.npz"), workload=np.array(w.name), **out)


def make_config4():
    w = config4()
    mesh, p = w.meshes[0], w.pulses[0][0]
    out = trajectory(mesh, p, w.h, w.steps, sample_nodes(mesh), log_every=50, tag=w.name)
    np.savez_compressed(os.path.join(HERE, "config4_rc_1024x1024_samples.npz"), workload=np.array(w.name), **out)


def make_config3b():
    """One grid of each side length of the 64-grid batch (the first of each), every step."""
    w = config3b()
    sides = [m.nx for m in w.meshes]
    grids = [sides.index(s) for s in sorted(set(sides))]
    res = {}
    nodes_all = []
    for g in grids:
        mesh = w.meshes[g]
        far = sample_nodes(mesh, n_random=0)
        nodes = sample_nodes(mesh, n_random=320 - far.size)
        nodes_all.append(nodes)
        o = trajectory(mesh, w.pulses[g][0], w.h, w.steps, nodes, log_every=100, tag=f"{w.name}[{g}]")
        for key in ("drops", "max_drop", "argmax", "sum_drop"):
            res.setdefault(key, []).append(o[key])
    np.savez_compressed(os.path.join(HERE, "config3b_batch_64grids_samples.npz"), workload=np.array(w.name),
                        grids=np.array(grids, np.int64), scenarios=np.zeros(len(grids), np.int64),
                        nodes=np.array(nodes_all), h=np.float64(w.h), vdd=np.float64(w.meshes[0].vdd),
                        steps=np.int64(w.steps), **{k: np.array(v) for k, v in res.items()})


def make_config4_adjoint(margin=0.05, rel_delta=1e-4, n_sample=4096):
    """The adjoint workload over its 200 steps: J, the oracle adjoint's gradient at seeded sampled
    entries of dJ/dC, dJ/dgE, dJ/dgN (and each gradient's largest magnitude), the directional
    derivative along ``workloads.random_direction`` from the oracle adjoint, and the same
    derivative by a central difference of the oracle's forward transient."""
    from dataclasses import replace
    from oracle import adjoint_gradients
    from oracle.adjoint import forward_states, softplus_loss
    w = config4()
    mesh, p = w.meshes[0], w.pulses[0][0]
    t0 = time.time()
    J, gC, gE, gN = adjoint_gradients(mesh, p, w.h, w.steps, margin)
    print(f"adjoint: J = {J:.12e} in {time.time() - t0:.1f} s", flush=True)
    dC, dE, dN = random_direction(mesh)
    dot = float(np.sum(gC * dC) + np.sum(gE * dE) + np.sum(gN * dN))

    def J_at(s):
        m = replace(mesh, C=mesh.C + s * dC, gE=mesh.gE + s * dE, gN=mesh.gN + s * dN)
        _, V = forward_states(m, p, w.h, w.steps)
        return softplus_loss(V[1:, : mesh.n], mesh.vdd, margin)

    fd = (J_at(rel_delta) - J_at(-rel_delta)) / (2 * rel_delta)
    print(f"directional: adjoint {dot:.12e}, central difference {fd:.12e} in {time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(np.random.SeedSequence(SAMPLE_SEED + 4))
    out = {}
    for name, g in (("C", gC), ("gE", gE), ("gN", gN)):
        idx = np.sort(rng.choice(g.size, size=n_sample, replace=False)).astype(np.int64)
        out[f"idx_{name}"] = idx
        out[f"grad_{name}"] = g.ravel()[idx]
        out[f"maxabs_{name}"] = np.float64(np.max(np.abs(g)))
    np.savez_compressed(os.path.join(HERE, "config4_adjoint_samples.npz"), workload=np.array(w.name),
                        J=np.float64(J), margin=np.float64(margin), steps=np.int64(w.steps),
                        dir_dot=np.float64(dot), dir_fd=np.float64(fd), rel_delta=np.float64(rel_delta), **out)


MAKERS = {"config0": make_config0, "config4_adjoint": make_config4_adjoint, "config1": make_config1, "config2": make_config2, "config3a": make_config3a,
          "config3b": make_config3b, "config4": make_config4}

if __name__ == "__main__":
    names = sys.argv[1:] or list(MAKERS)
    for name in names:
        MAKERS[name]()
