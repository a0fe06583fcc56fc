"""Pins of the oracle's Jacobi spectral radius, Young's relaxation factor and the
residual-to-error factor ||M^-1 D||_inf (closed forms, Young's theorem, brute force)."""
import numpy as np
import pytest

from oracle import BESystem, error_bound_factor, jacobi_radius, mesh_to_circuit, young_omega
from workloads import small_rc, small_multilayer, uniform_diagonal_mesh


def _step_matrix(w):
    circ, _ = mesh_to_circuit(w.meshes[0], None)
    return BESystem(circ, w.h).M


def _uniform(nx, ny, g=1.0, C=2e-12, h=1e-11):
    w = uniform_diagonal_mesh(nx, ny, g=g, C=C, h=h)
    c = C / h
    mu = lambda i, j: g * (2 * np.cos(np.pi * i / (nx + 1)) + 2 * np.cos(np.pi * j / (ny + 1))) / (c + 4 * g)
    return w, mu


@pytest.mark.parametrize("nx,ny", [(9, 6), (60, 40)])
def test_jacobi_radius_of_the_uniform_diagonal_grid(nx, ny):
    """J = g A / (C/h + 4g) with A the grid graph's adjacency, whose largest eigenvalue is
    2 cos(pi/(nx+1)) + 2 cos(pi/(ny+1)) (sine eigenvectors); the second size takes the sparse
    eigen-solver branch."""
    w, mu = _uniform(nx, ny)
    M = _step_matrix(w)
    d = M.diagonal()
    assert np.allclose(d, d[0], rtol=1e-14)
    assert jacobi_radius(M) == pytest.approx(mu(1, 1), rel=1e-10)


def _red_black_sor_radius(M, omega, colour):
    M = M.toarray()
    order = np.argsort(colour, kind="stable")
    A = M[np.ix_(order, order)]
    D = np.diag(np.diag(A))
    L = -np.tril(A, -1)
    U = -np.triu(A, 1)
    T = np.linalg.solve(D - omega * L, (1 - omega) * D + omega * U)
    return float(np.max(np.abs(np.linalg.eigvals(T))))


def test_young_omega_minimises_the_red_black_sor_radius():
    """Young's theorem for a consistently ordered matrix: at omega_opt the SOR matrix has
    spectral radius omega_opt - 1, and any other omega gives more."""
    w = small_rc(7, 6, seed=11, pad_every=3)
    mesh = w.meshes[0]
    M = _step_matrix(w)
    x, y = np.meshgrid(np.arange(mesh.nx), np.arange(mesh.ny))
    colour = ((x + y) & 1).ravel()
    rho = jacobi_radius(M)
    w_opt = young_omega(rho)
    r_opt = _red_black_sor_radius(M, w_opt, colour)
    assert r_opt == pytest.approx(w_opt - 1.0, abs=2e-4)
    for dw in (-0.03, 0.03):
        assert _red_black_sor_radius(M, w_opt + dw, colour) > r_opt + 1e-3


def test_error_bound_factor_of_the_uniform_diagonal_grid():
    """x = (I - J)^-1 1 summed over the sine eigenvectors, whose coefficients on the all-ones
    vector are known in closed form."""
    nx, ny = 11, 7
    w, mu = _uniform(nx, ny)
    M = _step_matrix(w)
    X = np.arange(nx)
    Y = np.arange(ny)
    x = np.zeros((ny, nx))
    for i in range(1, nx + 1):
        ux = np.sin(np.pi * i * (X + 1) / (nx + 1)) * np.sqrt(2.0 / (nx + 1))
        for j in range(1, ny + 1):
            uy = np.sin(np.pi * j * (Y + 1) / (ny + 1)) * np.sqrt(2.0 / (ny + 1))
            u = np.outer(uy, ux)
            x += u * (u.sum() / (1.0 - mu(i, j)))
    assert error_bound_factor(M) == pytest.approx(x.max(), rel=1e-12)


def test_error_bound_factor_by_brute_force_and_as_a_bound():
    w = small_multilayer(side=6, seed=12, nl=2, layer_g=(1.0, 2.0), pad_every=3)
    M = _step_matrix(w)
    A = M.toarray()
    Minv = np.linalg.inv(A)
    assert np.all(Minv > -1e-14)  # an M-matrix
    kappa = error_bound_factor(M)
    assert kappa == pytest.approx(np.max(np.abs(Minv * np.diag(A)[None, :]).sum(axis=1)), rel=1e-12)
    assert kappa >= 1.0
    rng = np.random.default_rng(1)
    b = rng.normal(size=A.shape[0])
    v = np.linalg.solve(A, b)
    for _ in range(20):
        vt = v + rng.normal(scale=1e-6, size=v.size)
        tau = np.max(np.abs(b - A @ vt) / np.diag(A))
        assert np.max(np.abs(vt - v)) <= kappa * tau * (1 + 1e-9)
