"""MI355X-native power-grid transient relaxation.

The hot path (right-hand side, red-black SOR sweeps on layered meshes or
colour-ordered sweeps on general netlists, FP64 residual and refinement,
inductor update) runs in the gfx950 kernels of ``libpgrid.so``;
``pgrid`` is its ctypes binding.  Build the library with
``python -m paper_1409_7166_amd.build``.
"""
from .pgrid import (Context, GraphShape, NetlistMesh, Options, PgError, default_options, lib, netlist_coloring,
                    netlist_to_mesh,
                    validate_mesh, validate_netlist, validate_options, PG_PREC_FP64, PG_PREC_FP32_REFINE,
                    PG_ORDER_RED_BLACK, PG_ORDER_JACOBI, PG_REC_TWO_LEVEL, PG_REC_THREE_LEVEL)

__all__ = ["Context", "GraphShape", "NetlistMesh", "Options", "PgError", "default_options", "lib",
           "netlist_coloring", "netlist_to_mesh",
           "validate_mesh", "validate_netlist", "validate_options", "PG_PREC_FP64", "PG_PREC_FP32_REFINE",
           "PG_ORDER_RED_BLACK", "PG_ORDER_JACOBI", "PG_REC_TWO_LEVEL", "PG_REC_THREE_LEVEL"]
