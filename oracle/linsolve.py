"""Direct solvers used as library primitives by the oracle (test infrastructure only).

Dense LU (LAPACK getrf via scipy) for small systems; SuperLU with a symmetric
minimum-degree ordering and no pivoting for larger ones (the system matrices
are symmetric positive definite by Lemma 1, so diagonal pivots are safe).
Indefinite systems (the DC saddle point with inductors) use SuperLU with
partial pivoting.

Parity: pinned by ``tests/test_oracle_rc.py::test_dense_and_sparse_solvers_agree`` (the
dense and the sparse factorisation give the same transient to 1e-13 V) and, through the
steppers that call it, by the closed-form and invariant tests of ``tests/test_oracle_rc.py``
and ``tests/test_oracle_rlc.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DENSE_MAX = 4096


class _Dense:
    def __init__(self, M):
        self.lu = sla.lu_factor(M.toarray() if sp.issparse(M) else np.asarray(M))

    def solve(self, b):
        return sla.lu_solve(self.lu, b)


class _Sparse:
    def __init__(self, M, spd):
        M = sp.csc_matrix(M)
        if spd:
            self.lu = spla.splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                                options=dict(SymmetricMode=True))
        else:
            self.lu = spla.splu(M)

    def solve(self, b):
        return self.lu.solve(np.asarray(b, float))


def factor(M, spd=True, dense_max=DENSE_MAX):
    """Factor M once; the returned object's ``solve(b)`` handles 1-D or 2-D ``b``."""
    n = M.shape[0]
    if n <= dense_max:
        return _Dense(M)
    return _Sparse(M, spd)
