"""Shared helpers for the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import sys

import torch  # noqa: F401  (first import can be slow on a fresh box; keep it out of test timeouts)

import numpy as np

import paper_1409_7166_amd as pg
from oracle import BEStepper, be_transient, mesh_to_circuit
from oracle.sources import currents_at
from workloads import Pulses

PARITY_V = 1e-6          # max |v_gpu - v_oracle| per node per step (volts)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_stream():
    import torch
    torch.cuda.set_device(0)
    return torch.cuda.current_stream().cuda_stream


def gpu_context(w, **opts):
    ctx = pg.Context(0, torch_stream())
    base = dict(h=w.h, tol=1e-10, omega=1.5, check_every=8, precision=pg.PG_PREC_FP64)
    base.update(opts)
    ctx.set_options(**base)
    for g, (mesh, scen) in enumerate(zip(w.meshes, w.pulses)):
        gid = ctx.upload_mesh(mesh, len(scen))
        assert gid == g
        for s, p in enumerate(scen):
            ctx.set_pulses(g, s, p)
    return ctx


def oracle_run(mesh, pulses, h, steps):
    circ, info = mesh_to_circuit(mesh, pulses)
    V, IL = be_transient(circ, info, pulses, h, steps)
    return V[:, : mesh.n], IL


def compressed(p, start=0.2, width=0.5, peak=1.0):
    """Pulses squeezed into an earlier, shorter window (same nodes)."""
    return Pulses(p.node, p.peak * peak, p.start * start, p.width * width)
