"""pg_update_mesh_values_dev (new segment conductances and capacitances from device memory,
coefficients rebuilt by kernels) against pg_update_mesh_values (host rebuild): the two must
give the same coefficients bit for bit, hence the same transient, for FP64 and FP32 sweeps,
RC and series R-L vias and pads, a zero supply, partial updates, updates that change which
layers carry capacitance, and a host update after a device one; bad values are refused with
nothing changed."""
import dataclasses

import numpy as np
import pytest
import torch

import paper_1409_7166_amd as pg
from helpers import gpu_context, say
from workloads import small_multilayer, small_rlc

pytestmark = pytest.mark.gpu


def _perturbed(mesh, seed, scale=0.3):
    r = np.random.default_rng(seed)
    f = lambda a: a * (1.0 + scale * r.uniform(-1, 1, a.shape))  # noqa: E731
    return f(mesh.gE), f(mesh.gN), f(mesh.C)


def _dev(a):
    return None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda:0")


def _run_pair(w, prec, updates, pre=4, post=20):
    """Two contexts stepped `pre` steps; then each update (gE, gN, C; None = unchanged) goes to
    context A through the host entry point and to context B through the device one."""
    opts = dict(precision=prec, tol=1e-11, omega=1.6, check_every=8)
    with gpu_context(w, **opts) as a, gpu_context(w, **opts) as b:
        a.step(pre)
        b.step(pre)
        for kind, (gE, gN, C) in updates:
            if kind == "host-both":
                a.update_mesh_values(0, gE, gN, C)
                b.update_mesh_values(0, gE, gN, C)
            else:
                a.update_mesh_values(0, gE, gN, C)
                b.update_mesh_values_dev(0, _dev(gE), _dev(gN), _dev(C))
            a.step(post // len(updates))
            b.step(post // len(updates))
        va, vb = a.read_voltages(), b.read_voltages()
        ia, ib = a.read_inductor_currents(), b.read_inductor_currents()
    return va, vb, ia, ib


@pytest.mark.parametrize("case", ["rc3-fp32", "rc3-fp64", "rlc2-fp32", "rlc2-fp64", "rc2-vdd0"])
def test_device_update_matches_host_update_bitwise(case):
    if case.startswith("rc3"):
        w = small_multilayer(side=72, seed=41, nl=3, pad_every=12, steps=40)
    elif case.startswith("rlc2"):
        w = small_rlc(side=48, seed=42, steps=40)
    else:
        w = small_multilayer(side=40, seed=43, nl=2, layer_g=(1.0, 4.0), pad_every=8, steps=40)
        w.meshes[0] = dataclasses.replace(w.meshes[0], vdd=0.0)
    prec = pg.PG_PREC_FP64 if case.endswith("fp64") else pg.PG_PREC_FP32_REFINE
    mesh = w.meshes[0]
    gE, gN, C = _perturbed(mesh, 7)
    gE2, _, C2 = _perturbed(mesh, 8)
    say(f"[gpu] device vs host coefficient update: {case}")
    va, vb, ia, ib = _run_pair(w, prec, [("dev", (gE, gN, C)), ("dev", (None, None, C2)), ("dev", (gE2, None, None))])
    assert np.array_equal(va, vb) and np.array_equal(ia, ib)
    assert np.max(np.abs(va - va.mean())) > 1e-5  # a loaded, non-trivial state


def test_layers_gaining_capacitance_and_a_later_host_update():
    w = small_multilayer(side=40, seed=44, nl=2, layer_g=(1.0, 4.0), pad_every=8, steps=40)
    mesh = w.meshes[0]
    gE, gN, C = _perturbed(mesh, 9)
    C_top = C.copy()
    C_top[1] = 2e-12  # the top layer had none: the set of layers with C/h changes
    say("[gpu] device update that gives a layer capacitance, then a partial host update")
    # A: host, host; B: device (falls back to a host rebuild), then host with only gE, which
    # must keep the device update's gN and C
    opts = dict(precision=pg.PG_PREC_FP32_REFINE, tol=1e-11, omega=1.6, check_every=8)
    with gpu_context(w, **opts) as a, gpu_context(w, **opts) as b:
        a.step(3)
        b.step(3)
        a.update_mesh_values(0, gE, gN, C_top)
        b.update_mesh_values_dev(0, _dev(gE), _dev(gN), _dev(C_top))
        a.step(6)
        b.step(6)
        gE3 = gE * 1.1
        a.update_mesh_values(0, gE3, None, None)
        b.update_mesh_values(0, gE3, None, None)
        a.step(6)
        b.step(6)
        assert np.array_equal(a.read_voltages(), b.read_voltages())


def test_bad_values_are_refused_and_change_nothing():
    w = small_multilayer(side=40, seed=45, nl=2, layer_g=(1.0, 4.0), pad_every=8, steps=40)
    mesh = w.meshes[0]
    gE, gN, C = _perturbed(mesh, 10)
    gN[1, 3, 7] = np.nan
    opts = dict(precision=pg.PG_PREC_FP64, tol=1e-11, omega=1.6, check_every=8)
    with gpu_context(w, **opts) as a, gpu_context(w, **opts) as b:
        a.step(3)
        b.step(3)
        with pytest.raises(pg.PgError) as ei:
            b.update_mesh_values_dev(0, _dev(gE), _dev(gN), _dev(C))
        assert ei.value.name == "PG_ERR_INVALID_ARG"
        bad = (1 * (mesh.ny - 1) + 3) * mesh.nx + 7
        assert f"gN[{bad}]" in str(ei.value)
        a.step(5)
        b.step(5)
        assert np.array_equal(a.read_voltages(), b.read_voltages())
        with pytest.raises(ValueError):
            b.update_mesh_values_dev(0, None, None, _dev(C[:, :-1]))
