"""FP64 CPU oracle for the power-grid transient (test infrastructure only).

This package is the reference the HIP path is checked against.  It is plain,
slow and written to be checked by eye against the paper
("An Efficient Topology-Based Algorithm for Transient Analysis of Power Grid",
Yang, Wang, Azevedo, Wang): it builds the incidence matrices of Sec. III
(eqs. 4-6), forms G, C, L, G_s, L_s (eq. 9, eq. 11), takes backward-Euler
steps (eqs. 2 and 10) by direct factorisation (dense LU for small systems,
SuperLU otherwise), derives the adjoint of the backward-Euler recurrence, and gives the
Jacobi spectral radius, Young's relaxation factor and the residual-to-error factor of a step
matrix.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  The product path never calls it, and it shares no
code, constant or helper with the HIP library: the only common input is the
seeded workload arrays from ``workloads``.

Parity status per function is listed in the module headers.
"""
from .circuit import Circuit, GROUND, mesh_to_circuit
from .sources import triangle_current, currents_at
from .linsolve import factor
from .transient import (BESystem, BEStepper, be_transient, dc_solve, three_level_transient,
                        scaled_residual, mesh_voltages)
from .adjoint import softplus_loss, adjoint_gradients, tangent_linear
from .spectral import jacobi_radius, young_omega, error_bound_factor

__all__ = ["Circuit", "GROUND", "mesh_to_circuit", "triangle_current", "currents_at",
           "factor", "BESystem", "BEStepper", "be_transient", "dc_solve", "three_level_transient",
           "scaled_residual", "mesh_voltages", "softplus_loss", "adjoint_gradients",
           "tangent_linear", "jacobi_radius", "young_omega", "error_bound_factor"]
