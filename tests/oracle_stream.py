"""Oracle trajectories computed in worker processes and handed to a GPU test step by step
(test infrastructure).

A long parity test cannot keep a whole oracle trajectory (a 256-scenario batch over 500 steps is
67 GB in FP64), and a single process cannot afford the oracle's direct solves for every item of a
batch one after another.  ``OracleStream`` runs a generator of per-step oracle states in a spawned
worker process (which imports only ``oracle``, ``workloads`` and numpy: no GPU, no torch) and a
thread of the test process receives the states into a short queue, so the oracle runs ahead of the
GPU comparison by a few steps while several workers share a batch.

Every state here comes from ``oracle.BEStepper`` (eq. 2 for RC meshes, eq. 10 in companion form
for series R-L vias and pads), from v = vdd and zero inductor current at t = 0.
"""
from __future__ import annotations

import multiprocessing as mp
import queue
import threading

import numpy as np


def build_workload(spec):
    """``spec`` = (generator name in ``workloads``, keyword arguments)."""
    import workloads
    name, kwargs = spec
    return getattr(workloads, name)(**kwargs)


def mesh_trajectory(spec, items, steps, every=1, currents=False):
    """Yield ``(k, [v_mesh of each item], [i_l of each item] or None)`` for k = every, 2 every, ..
    ``items`` = [(grid, scenario), ...]; the oracle factors each grid's step matrix once."""
    from oracle import BEStepper, mesh_to_circuit
    from oracle.sources import currents_at
    from oracle.transient import initial_state

    w = build_workload(spec)
    steppers, state, n_mesh, init = {}, {}, {}, {}
    for g, s in items:
        mesh, p = w.meshes[g], w.pulses[g][s]
        if g not in steppers:
            circ, info = mesh_to_circuit(mesh, p)
            steppers[g] = BEStepper(circ, w.h)
            n_mesh[g] = info["n_mesh"]
            init[g] = initial_state(circ, info, mesh.vdd)
        state[(g, s)] = (init[g][0].copy(), init[g][1].copy())
    for k in range(1, steps + 1):
        for g, s in items:
            v, il = state[(g, s)]
            state[(g, s)] = steppers[g].step(v, il, currents_at(w.pulses[g][s], k * w.h))
        if k % every == 0:
            vs = [state[it][0][: n_mesh[it[0]]].copy() for it in items]
            ils = [state[it][1].copy() for it in items] if currents else None
            yield k, vs, ils


def _run(conn, fn_name, args):
    fn = globals()[fn_name]
    try:
        for item in fn(*args):
            conn.send(("step", item))
        conn.send(("done", None))
    except BaseException as e:  # noqa: BLE001 - reported to the test
        conn.send(("error", repr(e)))
    finally:
        conn.close()


class OracleStream:
    """Run ``fn_name(*args)`` (a generator in this module) in a spawned worker; ``get()`` returns
    its next item.  At most ``depth`` items wait in the test process."""

    def __init__(self, fn_name, args, depth=4):
        ctx = mp.get_context("spawn")
        recv, send = ctx.Pipe(duplex=False)
        self.proc = ctx.Process(target=_run, args=(send, fn_name, args), daemon=True)
        self.proc.start()
        send.close()
        self.q = queue.Queue(maxsize=depth)
        self.thread = threading.Thread(target=self._drain, args=(recv,), daemon=True)
        self.thread.start()

    def _drain(self, recv):
        while True:
            try:
                msg = recv.recv()
            except (EOFError, OSError):
                self.q.put(("error", "oracle worker ended without a result"))
                return
            self.q.put(msg)
            if msg[0] != "step":
                return

    def get(self, timeout=900):
        tag, val = self.q.get(timeout=timeout)
        if tag == "error":
            raise RuntimeError(f"oracle worker failed: {val}")
        if tag == "done":
            raise StopIteration
        return val

    def close(self):
        if self.proc.is_alive():
            self.proc.terminate()
        self.proc.join(timeout=10)


class BatchStream:
    """Several ``mesh_trajectory`` workers over disjoint item lists of one workload; ``get()``
    returns ``(k, {item: v}, {item: i_l} or None)`` merged over the workers."""

    def __init__(self, spec, chunks, steps, every=1, currents=False, depth=3):
        self.chunks = [list(c) for c in chunks if len(c)]
        self.streams = [OracleStream("mesh_trajectory", (spec, c, steps, every, currents), depth)
                        for c in self.chunks]

    def get(self, timeout=900):
        vs, ils, k0 = {}, {}, None
        for chunk, st in zip(self.chunks, self.streams):
            k, v, il = st.get(timeout)
            assert k0 is None or k == k0
            k0 = k
            vs.update(zip(chunk, v))
            if il is not None:
                ils.update(zip(chunk, il))
        return k0, vs, (ils or None)

    def close(self):
        for st in self.streams:
            st.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def balanced_chunks(items, weights, n):
    """Split ``items`` into at most ``n`` lists of similar total weight (largest first)."""
    order = np.argsort(-np.asarray(weights, float), kind="stable")
    bins = [[] for _ in range(n)]
    load = np.zeros(n)
    for i in order:
        j = int(np.argmin(load))
        bins[j].append(items[i])
        load[j] += weights[i]
    return [sorted(b) for b in bins if b]
