"""Backward-Euler transient, DC operating point and the three-level recurrence
(test infrastructure only).

Parity: pinned.  ``tests/test_oracle_rc.py`` and ``tests/test_oracle_rlc.py``
check these functions against closed forms (single RC node, uniform mesh
diagonalised by the DCT, hand-solved two-node and R-L tank circuits),
invariants (Vdd fixed point, superposition, charge balance, maximum principle,
reciprocity, energy decay) and against each other (two-level vs three-level,
transient vs DC).

Conventions (Sec. III, signs as derived in ``oracle.circuit``):
  node equation      C dv/dt + G v + A_l^T i_l + A_i^T I_s + G_s v_d = 0
  inductor equation  L di_l/dt - A_l v - A_ls v_d = 0
Backward Euler (eq. 10) with step h, eliminating i_l(t+h):
  (C/h + G + h L) v(t+h) = (C/h) v(t) - A_l^T i_l(t) - h L_s v_d
                           - A_i^T I_s(t+h) - G_s v_d
  i_l(t+h) = i_l(t) + h L^-1 (A_l v(t+h) + A_ls v_d)
For an RC circuit this is eq. 2 with b(t+h) = -i(t+h) + G0 Vdd, because
-G_s v_d is the pad injection G0 Vdd.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .linsolve import factor
from .sources import currents_at


class BESystem:
    """The assembled backward-Euler system of eq. 10 (system matrix and right-hand side)."""

    def __init__(self, circ, h: float):
        self.circ = circ
        self.h = float(h)
        mats = circ.matrices()
        self.mats = mats
        self.Ch = (mats["C"] / self.h).tocsr()
        self.M = (self.Ch + mats["G"] + self.h * mats["L"]).tocsc()
        vd = circ.vd
        # constant part of the right-hand side: -h L_s v_d - G_s v_d
        self.const = -(self.h * (mats["Ls"] @ vd)) - (mats["Gs"] @ vd)
        self.Linv = 1.0 / mats["Lvals"] if mats["Lvals"].size else np.zeros(0)

    def rhs(self, v, il, I_next):
        mats = self.mats
        b = self.Ch @ v + self.const
        if il.size:
            b = b - mats["Al"].T @ il
        if I_next.size:
            b = b - mats["Ai"].T @ I_next
        return b


class BEStepper(BESystem):
    """One backward-Euler step of eq. 10 with the system matrix factored once."""

    def __init__(self, circ, h: float, dense_max: int | None = None):
        super().__init__(circ, h)
        kw = {} if dense_max is None else {"dense_max": dense_max}
        self.fac = factor(self.M, spd=True, **kw)

    def step(self, v, il, I_next):
        b = self.rhs(v, il, I_next)
        v1 = self.fac.solve(b)
        il1 = il
        if il.size:
            mats = self.mats
            il1 = il + self.h * self.Linv * (mats["Al"] @ v1 + mats["Als"] @ self.circ.vd)
        return v1, il1


def initial_state(circ, info, vdd):
    """All trivial nodes at the supply voltage and no inductor current.

    This is the DC operating point whenever no source draws current at t = 0,
    which holds for every triangular pulse with a non-negative start.
    """
    n_l = int(np.sum(circ.kind == "L"))
    return np.full(circ.n, float(vdd)), np.zeros(n_l)


def mesh_voltages(v, info):
    return v[: info["n_mesh"]]


def be_transient(circ, info, pulses, h, steps, v0=None, il0=None, callback=None,
                 store=True, dense_max=None):
    """Run ``steps`` backward-Euler steps from (v0, il0) at t = 0.

    Step k (1-based) uses the sources at t_k = k h.  Returns (V, IL) with the
    trivial-node voltages and inductor currents after every step when ``store``;
    ``callback(k, v, il)`` is called after every step either way.
    """
    st = BEStepper(circ, h, dense_max=dense_max)
    if v0 is None or il0 is None:
        v_init, il_init = initial_state(circ, info, circ.vd[0])
        v0 = v_init if v0 is None else v0
        il0 = il_init if il0 is None else il0
    v, il = np.array(v0, float), np.array(il0, float)
    V, IL = [], []
    for k in range(1, steps + 1):
        v, il = st.step(v, il, currents_at(pulses, k * h))
        if store:
            V.append(v.copy()); IL.append(il.copy())
        if callback is not None:
            callback(k, v, il)
    if store:
        return np.array(V), np.array(IL)
    return v, il


def dc_solve(circ, I_now):
    """DC operating point for source currents I_now (eq. 3 with A = G, inductors shorted).

    Capacitors carry no current; each inductor is a short, so its voltage is zero:
      G v + A_l^T i_l = -A_i^T I - G_s v_d,    A_l v = -A_ls v_d.
    Returns (v, i_l).
    """
    mats = circ.matrices()
    vd = circ.vd
    b = -(mats["Gs"] @ vd)
    if I_now.size:
        b = b - mats["Ai"].T @ I_now
    nl = mats["Al"].shape[0]
    if nl == 0:
        v = factor(mats["G"].tocsc(), spd=True).solve(b)
        return v, np.zeros(0)
    K = sp.bmat([[mats["G"], mats["Al"].T], [mats["Al"], None]]).tocsc()
    rhs = np.concatenate([b, -(mats["Als"] @ vd)])
    x = factor(K, spd=False, dense_max=0).solve(rhs)
    return x[: circ.n], x[circ.n:]


def three_level_transient(circ, pulses, h, steps, v0, v1):
    """The paper's three-level recurrence (eq. 11), seeded with v(0) and v(h).

    (C/h + G + h L) v(t+h) = (2C/h + G) v(t) - (C/h) v(t-h) - h L_s v_d
                             - A_i^T (I_s(t+h) - I_s(t))
    Returns the voltages for steps 2..steps (index 0 is step 2).
    """
    mats = circ.matrices()
    Ch = mats["C"] / h
    M = (Ch + mats["G"] + h * mats["L"]).tocsc()
    fac = factor(M, spd=True)
    R1 = (2.0 * Ch + mats["G"]).tocsr()
    c = -(h * (mats["Ls"] @ circ.vd))
    vm, v = np.array(v0, float), np.array(v1, float)
    out = []
    for k in range(2, steps + 1):
        dI = currents_at(pulses, k * h) - currents_at(pulses, (k - 1) * h)
        b = R1 @ v - Ch @ vm + c
        if dI.size:
            b = b - mats["Ai"].T @ dI
        vm, v = v, fac.solve(b)
        out.append(v.copy())
    return np.array(out)


def scaled_residual(stepper: BESystem, v_prev, il_prev, v_next, I_next):
    """max_i |(b - M v_next)_i| / M_ii, the Jacobi-scaled backward-Euler residual (volts)."""
    b = stepper.rhs(v_prev, il_prev, I_next)
    r = b - stepper.M @ v_next
    return float(np.max(np.abs(r) / stepper.M.diagonal()))
