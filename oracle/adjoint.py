"""Reverse-time adjoint and tangent-linear of the RC backward-Euler transient
(test infrastructure only).

Parity: pinned by ``tests/test_oracle_adjoint.py``: per-parameter central
finite differences of the oracle's own forward transient on small meshes, and
the tangent-linear / adjoint dot-product identity.

The forward recurrence is eq. 2 on a layered mesh: M v_k = (C/h) v_{k-1} + f_k,
M = C/h + G (G includes the pad conductances), f_k = G0 Vdd - i(t_k), k = 1..K,
v_0 = Vdd.  The loss is J = sum_{k=1..K} sum_i softplus(Vdd - v_{k,i} - margin)^2.
With lambda_{K+1} = 0 the adjoint recurrence (M symmetric by Lemma 1) is
  M lambda_k = dJ/dv_k + (C/h) lambda_{k+1},
and the gradients with respect to a node capacitance C_i and a mesh segment
conductance g_e between nodes a and b are
  dJ/dC_i = sum_k lambda_{k,i} (v_{k-1,i} - v_{k,i}) / h,
  dJ/dg_e = - sum_k (lambda_{k,a} - lambda_{k,b}) (v_{k,a} - v_{k,b}).
A via is such a branch between (x, y, l) and (x, y, l+1); a pad of conductance g_p at node a
adds g_p to M_aa and g_p Vdd to f_k, so
  dJ/dg_p = sum_k lambda_{k,a} (Vdd - v_{k,a}).
Source waveforms are held fixed.
"""
from __future__ import annotations

import numpy as np

from .circuit import mesh_to_circuit
from .sources import currents_at
from .transient import BEStepper


def _softplus(x):
    return np.logaddexp(0.0, x)


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def softplus_loss(V, vdd, margin):
    """J over a stack of mesh-voltage vectors (steps 1..K)."""
    u = vdd - np.asarray(V) - margin
    return float(np.sum(_softplus(u) ** 2))


def _dloss(v, vdd, margin):
    u = vdd - v - margin
    return -2.0 * _softplus(u) * _sigmoid(u)


def _edges(mesh):
    ids = np.arange(mesh.n).reshape(mesh.nl, mesh.ny, mesh.nx)
    return (ids[:, :, :-1], ids[:, :, 1:]), (ids[:, :-1, :], ids[:, 1:, :])


def forward_states(mesh, pulses, h, steps):
    circ, info = mesh_to_circuit(mesh, pulses)
    if np.any(circ.kind == "L"):
        raise ValueError("the adjoint oracle covers RC meshes only")
    st = BEStepper(circ, h)
    V = np.empty((steps + 1, circ.n))
    V[0] = mesh.vdd
    il = np.zeros(0)
    for k in range(1, steps + 1):
        V[k], _ = st.step(V[k - 1], il, currents_at(pulses, k * h))
    return st, V


def adjoint_gradients(mesh, pulses, h, steps, margin):
    """Return (J, dJ/dC [nl,ny,nx], dJ/dgE [nl,ny,nx-1], dJ/dgN [nl,ny-1,nx])."""
    return _adjoint(mesh, pulses, h, steps, margin)[:4]


def adjoint_branch_gradients(mesh, pulses, h, steps, margin):
    """Return (dJ/dvia_g [n_vias], dJ/dpad_g [n_pads]) in the mesh's via and pad order."""
    return _adjoint(mesh, pulses, h, steps, margin)[4:]


def _adjoint(mesh, pulses, h, steps, margin):
    st, V = forward_states(mesh, pulses, h, steps)
    vdd = mesh.vdd
    J = softplus_loss(V[1:], vdd, margin)
    (ea, eb), (na, nb) = _edges(mesh)
    dC = np.zeros(mesh.n)
    dgE = np.zeros(ea.shape)
    dgN = np.zeros(na.shape)
    va = np.asarray(mesh.via_node, np.int64); vb = va + mesh.nx * mesh.ny
    pa = np.asarray(mesh.pad_node, np.int64)
    dvia = np.zeros(va.size)
    dpad = np.zeros(pa.size)
    lam_next = np.zeros(mesh.n)
    for k in range(steps, 0, -1):
        lam = st.fac.solve(_dloss(V[k], vdd, margin) + st.Ch @ lam_next)
        vk = V[k]
        dC += lam * (V[k - 1] - vk) / h
        dgE -= (lam[ea] - lam[eb]) * (vk[ea] - vk[eb])
        dgN -= (lam[na] - lam[nb]) * (vk[na] - vk[nb])
        dvia -= (lam[va] - lam[vb]) * (vk[va] - vk[vb])
        dpad += lam[pa] * (vdd - vk[pa])
        lam_next = lam
    shape = (mesh.nl, mesh.ny, mesh.nx)
    return J, dC.reshape(shape), dgE, dgN, dvia, dpad


def tangent_linear(mesh, pulses, h, steps, margin, dC, dgE, dgN):
    """Directional derivative dJ . (dC, dgE, dgN) by forward sensitivities.

    Differentiating M v_k = (C/h) v_{k-1} + f_k gives
      M dv_k = (dC/h) (v_{k-1} - v_k) - dG v_k + (C/h) dv_{k-1},  dv_0 = 0,
    and dJ = sum_k (dJ/dv_k) . dv_k.
    """
    st, V = forward_states(mesh, pulses, h, steps)
    (ea, eb), (na, nb) = _edges(mesh)
    dC = np.asarray(dC).ravel()
    dv = np.zeros(mesh.n)
    total = 0.0
    for k in range(1, steps + 1):
        vk = V[k]
        dGv = np.zeros(mesh.n)
        for (a, b), dg in (((ea, eb), dgE), ((na, nb), dgN)):
            f = dg * (vk[a] - vk[b])
            np.add.at(dGv, a.ravel(), f.ravel())
            np.add.at(dGv, b.ravel(), -f.ravel())
        rhs = dC / h * (V[k - 1] - vk) - dGv + st.Ch @ dv
        dv = st.fac.solve(rhs)
        total += float(_dloss(vk, mesh.vdd, margin) @ dv)
    return total
