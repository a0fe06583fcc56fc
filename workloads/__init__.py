"""Seeded synthetic power-grid workloads shared by the oracle, the tests and the bench.

This package only draws random circuit parameters and lays them out as plain
arrays (mesh conductances, capacitances, vias, pads, current pulses).  It holds
none of the transient method's arithmetic: no matrix assembly, no time
stepping, no solver.  Both the CPU oracle and the HIP path consume the same
arrays, so any disagreement between them comes from the method, not the inputs.
"""
from .grids import (Mesh, Pulses, Workload, config0, config1, config2, config3a, random_mesh, random_direction,
                    config3b, config4, small_rc, small_rlc, small_multilayer,
                    uniform_diagonal_mesh, pulse_draw, CONFIGS)
from .netlists import Netlist, NetWorkload, graph1, graph_mesh1, irregular_grid, mesh_netlist

__all__ = ["Mesh", "Pulses", "Workload", "config0", "config1", "config2",
           "config3a", "config3b", "config4", "small_rc", "small_rlc",
           "small_multilayer", "uniform_diagonal_mesh", "pulse_draw", "CONFIGS", "random_mesh", "random_direction",
           "Netlist", "NetWorkload", "graph1", "graph_mesh1", "irregular_grid", "mesh_netlist"]
