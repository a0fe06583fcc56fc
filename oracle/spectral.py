"""Jacobi spectral radius, Young's relaxation factor and the residual-to-error factor
(test infrastructure only).

Parity: pinned.  ``tests/test_oracle_spectral.py`` checks these functions against closed forms
on a grid whose diagonal is uniform (its Jacobi matrix is a multiple of the grid graph's
adjacency, diagonalised by sine vectors), against Young's theorem (the red-black SOR iteration
matrix has spectral radius omega_opt - 1 at omega_opt and more on either side), and against
dense brute force on tiny systems.

For an SPD M with diagonal D (Lemma 1):
  Jacobi iteration matrix   J = I - D^-1 M, similar to S = D^-1/2 (D - M) D^-1/2 (symmetric);
  rho_J = max |eig(S)|;
  Young's optimum for a consistently ordered matrix (eq. 17's omega with red-black ordering)
    omega_opt = 2 / (1 + sqrt(1 - rho_J^2));
  ||M^-1 D||_inf = max_i (M^-1 D 1)_i when M^-1 >= 0 entrywise (an M-matrix), so a scaled
    residual max_i |r_i| / M_ii <= tau bounds the error of M v = b by ||M^-1 D||_inf * tau.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .linsolve import factor


def jacobi_radius(M) -> float:
    """rho(I - D^-1 M) via the symmetric similar matrix D^-1/2 (D - M) D^-1/2."""
    M = sp.csr_matrix(M)
    d = M.diagonal()
    s = 1.0 / np.sqrt(d)
    S = sp.diags(s) @ (sp.diags(d) - M) @ sp.diags(s)
    n = M.shape[0]
    if n <= 2000:
        ev = np.linalg.eigvalsh(S.toarray())
        return float(np.max(np.abs(ev)))
    hi = spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-12)[0]
    lo = spla.eigsh(S, k=1, which="SA", return_eigenvectors=False, tol=1e-12)[0]
    return float(max(abs(hi), abs(lo)))


def young_omega(rho: float) -> float:
    return 2.0 / (1.0 + np.sqrt(1.0 - rho * rho))


def error_bound_factor(M) -> float:
    """max_i (M^-1 D 1)_i."""
    M = sp.csc_matrix(M)
    x = factor(M, spd=True).solve(M.diagonal())
    return float(np.max(x))
