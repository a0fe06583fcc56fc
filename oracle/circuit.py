"""Circuit description and the matrices of the paper's nodal formulation (Sec. III).

Parity: pinned (closed forms, invariants and hand-worked examples in
``tests/test_oracle_*.py``).

Nodes follow the paper's split: ``n`` trivial nodes (unknown voltages) and
``p`` source nodes (positive terminals of ideal supplies whose negative
terminals are grounded, assumption 1).  Branch endpoints are encoded as
  * ``0 .. n-1``       trivial node,
  * ``n .. n+p-1``     source node ``j = code - n``,
  * ``GROUND`` (-1)    ground.
Branch kinds: 'R' (value = conductance, S), 'C' (capacitance, F),
'L' (inductance, H), 'I' (current source; value = index into the source table).
Branch current flows from ``frm`` to ``to``.

Sign reading: the branch-voltage law is v_b = A v_n + A_s v_d (KVL of eq. 7);
substituted into the branch laws (eq. 8) and KCL, the node equation becomes
C dv/dt + G v + A_l^T i_l + A_i^T I_s + G_s v_d = 0 and the inductor equation
L di_l/dt - A_l v - A_ls v_d = 0.  Eq. 9 prints the v_d terms with the opposite
sign; the signs used here are the ones that make a pad pull its node towards
the supply voltage.  The diagonal matrix in eq. 8 holds conductances.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

GROUND = -1


@dataclass
class Circuit:
    n: int
    vd: np.ndarray          # (p,) source voltages
    frm: np.ndarray         # (m,) int64 endpoint codes
    to: np.ndarray          # (m,)
    kind: np.ndarray        # (m,) '<U1'
    value: np.ndarray       # (m,) float64

    @property
    def p(self) -> int:
        return int(self.vd.size)

    @property
    def m(self) -> int:
        return int(self.frm.size)

    # --- eq. 4 and eq. 5: modified incidence and source incidence ------------------
    def incidence(self):
        """Return (A, A_s): A is m x n over trivial nodes, A_s is m x p over source nodes.

        Entry +1 where the node is the branch's source terminal (``frm``), -1 where
        it is the sink (``to``), 0 otherwise; ground has no column.
        """
        m, n, p = self.m, self.n, self.p
        rows, cols, vals = [], [], []
        srows, scols, svals = [], [], []
        for end, sign in ((self.frm, 1.0), (self.to, -1.0)):
            triv = (end >= 0) & (end < n)
            src = end >= n
            rows.append(np.nonzero(triv)[0]); cols.append(end[triv]); vals.append(np.full(triv.sum(), sign))
            srows.append(np.nonzero(src)[0]); scols.append(end[src] - n); svals.append(np.full(src.sum(), sign))
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
        As = sp.csr_matrix((np.concatenate(svals), (np.concatenate(srows), np.concatenate(scols))), shape=(m, p))
        return A, As

    # --- eq. 6: grouping by element kind ---------------------------------------------
    def grouped(self):
        """Return dict kind -> (rows of A, rows of A_s, branch values, branch indices)."""
        A, As = self.incidence()
        out = {}
        for k in "RCLI":
            idx = np.nonzero(self.kind == k)[0]
            out[k] = (A[idx], As[idx], self.value[idx], idx)
        return out

    # --- eq. 9 and eq. 11: the reduced matrices ------------------------------------------
    def matrices(self):
        """G = A_g^T Gd A_g, C = A_c^T Cd A_c, G_s = A_g^T Gd A_gs, L = A_l^T Ld^-1 A_l,
        L_s = A_l^T Ld^-1 A_ls, and A_i (for the current-source injection A_i^T I_s)."""
        g = self.grouped()
        Ag, Ags, gv, _ = g["R"]
        Ac, _, cv, _ = g["C"]
        Al, Als, lv, _ = g["L"]
        Ai, _, _, _ = g["I"]
        Gd = sp.diags(gv)
        Cd = sp.diags(cv)
        Linv = sp.diags(1.0 / lv) if lv.size else sp.diags(np.zeros(0))
        G = (Ag.T @ Gd @ Ag).tocsr()
        C = (Ac.T @ Cd @ Ac).tocsr()
        Gs = (Ag.T @ Gd @ Ags).tocsr()
        L = (Al.T @ Linv @ Al).tocsr()
        Ls = (Al.T @ Linv @ Als).tocsr()
        return dict(G=G, C=C, Gs=Gs, L=L, Ls=Ls, Al=Al.tocsr(), Als=Als.tocsr(), Ai=Ai.tocsr(),
                    Lvals=lv, L_index=g["L"][3], I_index=g["I"][3])

    def system_matrix(self, h: float):
        """M = C/h + G + h L (eq. 11); for RC circuits M = C/h + G (eq. 2)."""
        mats = self.matrices()
        return (mats["C"] / h + mats["G"] + h * mats["L"]).tocsc()


def mesh_to_circuit(mesh, pulses=None):
    """Translate a layered mesh (see ``workloads.grids``) into the paper's branch list.

    Trivial nodes ``0 .. mesh.n-1`` are the mesh nodes; a series R-L via or pad
    adds one internal trivial node between its resistor and its inductor.  A
    single source node holds ``mesh.vdd``.  Each pulse becomes a current-source
    branch from its node to ground, numbered in pulse order.

    Returns (circuit, info) where ``info['n_mesh']`` is the number of mesh nodes.
    """
    nx, ny, nl = mesh.nx, mesh.ny, mesh.nl
    ids = np.arange(mesh.n, dtype=np.int64).reshape(nl, ny, nx)
    frm, to, kind, val = [], [], [], []

    def add(a, b, k, v):
        a = np.asarray(a, np.int64).ravel(); b = np.asarray(b, np.int64).ravel()
        v = np.broadcast_to(np.asarray(v, float).ravel(), a.shape)
        frm.append(a); to.append(b); kind.append(np.full(a.size, k)); val.append(np.array(v))

    # metal segments (resistors)
    add(ids[:, :, :-1], ids[:, :, 1:], "R", mesh.gE)
    add(ids[:, :-1, :], ids[:, 1:, :], "R", mesh.gN)
    # decaps to ground
    cmask = mesh.C.ravel() > 0
    add(ids.ravel()[cmask], np.full(cmask.sum(), GROUND), "C", mesh.C.ravel()[cmask])

    n_mesh = mesh.n
    src = -2  # placeholder for the supply node's code, fixed once n is known
    # vias: lower-layer node -> upper-layer node; pads: node -> supply.
    # A branch with L > 0 is split into R (node -> internal node q) and L (q -> far end).
    lo = mesh.via_node.astype(np.int64)
    far = [lo + nx * ny, np.full(mesh.pad_node.size, src, np.int64)]
    near = [lo, mesh.pad_node.astype(np.int64)]
    gval = [mesh.via_g, mesh.pad_g]
    lval = [mesh.via_L, mesh.pad_L]
    n_extra = 0
    internal = {}
    for name, a, b, gv, lv in zip(("via", "pad"), near, far, gval, lval):
        ind = lv > 0
        add(a[~ind], b[~ind], "R", gv[~ind])
        q = n_mesh + n_extra + np.arange(ind.sum(), dtype=np.int64)
        n_extra += int(ind.sum())
        add(a[ind], q, "R", gv[ind])
        add(q, b[ind], "L", lv[ind])
        internal[name] = (np.nonzero(ind)[0], q)
    if pulses is not None and pulses.count:
        add(pulses.node, np.full(pulses.count, GROUND), "I", np.arange(pulses.count, dtype=float))

    n = n_mesh + n_extra
    frm = np.concatenate(frm); to = np.concatenate(to)
    frm[frm == src] = n
    to[to == src] = n
    circ = Circuit(n=n, vd=np.array([mesh.vdd], float), frm=frm, to=to,
                   kind=np.concatenate(kind), value=np.concatenate(val))
    return circ, {"n_mesh": n_mesh, "internal": internal}
