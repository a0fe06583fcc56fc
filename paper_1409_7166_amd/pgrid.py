"""ctypes binding of ``libpgrid.so`` (the C ABI declared in ``include/pgrid.h``).

Argument marshalling only: every step of the transient runs in the library's HIP
kernels.  Host arrays are passed as contiguous numpy buffers; device outputs can
be torch tensors on the context's device, whose stream the context may share.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpgrid.so")

PG_PREC_FP64 = 0
PG_PREC_FP32_REFINE = 1
PG_ORDER_RED_BLACK = 0
PG_ORDER_JACOBI = 1
PG_REC_TWO_LEVEL = 0
PG_REC_THREE_LEVEL = 1

STATUS = {0: "PG_OK", -1: "PG_ERR_INVALID_ARG", -2: "PG_ERR_TOPOLOGY", -3: "PG_ERR_NOT_SPD",
          -4: "PG_ERR_NO_CONVERGENCE", -5: "PG_ERR_DEVICE", -6: "PG_ERR_OOM", -7: "PG_ERR_STATE",
          -8: "PG_ERR_UNSUPPORTED"}


class PgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Options(C.Structure):
    _fields_ = [("h", C.c_double), ("tol", C.c_double), ("omega", C.c_double),
                ("max_sweeps", C.c_int32), ("check_every", C.c_int32), ("precision", C.c_int32),
                ("ordering", C.c_int32), ("tile_rows", C.c_int32), ("lookahead", C.c_int32),
                ("graphs", C.c_int32), ("scen_block", C.c_int32),
                ("sweeps_per_launch", C.c_int32), ("recurrence", C.c_int32), ("resident", C.c_int32),
                ("predictor", C.c_int32)]


class MeshStruct(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nl", C.c_int32),
                ("gE", C.POINTER(C.c_double)), ("gN", C.POINTER(C.c_double)), ("C", C.POINTER(C.c_double)),
                ("n_vias", C.c_int32), ("via_node", C.POINTER(C.c_int32)), ("via_g", C.POINTER(C.c_double)),
                ("via_L", C.POINTER(C.c_double)),
                ("n_pads", C.c_int32), ("pad_node", C.POINTER(C.c_int32)), ("pad_g", C.POINTER(C.c_double)),
                ("pad_L", C.POINTER(C.c_double)), ("vdd", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("sweeps", C.c_int64), ("node_updates", C.c_int64),
                ("checks", C.c_int64), ("last_step_sweeps", C.c_int32), ("max_step_sweeps", C.c_int32),
                ("last_residual", C.c_double), ("max_final_residual", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelTimes(C.Structure):
    _fields_ = [("sweep_launches", C.c_int64), ("sweep_ms", C.c_double), ("sweep_node_updates", C.c_int64),
                ("sweep_bytes", C.c_double),
                ("resid_launches", C.c_int64), ("resid_ms", C.c_double), ("resid_nodes", C.c_int64),
                ("resid_bytes", C.c_double),
                ("rhs_launches", C.c_int64), ("rhs_ms", C.c_double),
                ("other_launches", C.c_int64), ("other_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_VOIDP = C.c_void_p  # (methods whose capacitance argument is named C shadow the module)

EXPORTS = {
    "pg_abi_version": (C.c_int32, []),
    "pg_status_name": (C.c_char_p, [C.c_int32]),
    "pg_default_options": (C.c_int, [C.POINTER(Options)]),
    "pg_validate_options": (C.c_int, [C.POINTER(Options), C.c_char_p, C.c_size_t]),
    "pg_validate_mesh": (C.c_int, [C.POINTER(MeshStruct), C.c_char_p, C.c_size_t]),
    "pg_validate_netlist": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_uint8), C.POINTER(C.c_double),
                                      C.c_char_p, C.c_size_t]),
    "pg_netlist_mesh_counts": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_uint8),
                                         C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.c_char_p, C.c_size_t]),
    "pg_netlist_to_mesh": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_uint8),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.c_char_p, C.c_size_t]),
    "pg_netlist_coloring": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_uint8),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_char_p, C.c_size_t]),
    "pg_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    "pg_destroy": (None, [C.c_void_p]),
    "pg_last_error": (C.c_char_p, [C.c_void_p]),
    "pg_set_options": (C.c_int, [C.c_void_p, C.POINTER(Options)]),
    "pg_get_options": (C.c_int, [C.c_void_p, C.POINTER(Options)]),
    "pg_upload_mesh": (C.c_int, [C.c_void_p, C.POINTER(MeshStruct), C.c_int32, C.POINTER(C.c_int32)]),
    "pg_upload_netlist": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_uint8),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32,
                                    C.POINTER(C.c_int32)]),
    "pg_set_pulses": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pg_set_pwl": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pg_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pg_reset": (C.c_int, [C.c_void_p]),
    "pg_dc_operating_point": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_int32]),
    "pg_estimate_omega": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "pg_error_bound_factor": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "pg_error_bound_factor_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "pg_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "pg_step_enqueue": (C.c_int, [C.c_void_p, C.c_int32]),
    "pg_run_transient": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(C.c_double)]),
    "pg_get_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pg_set_time": (C.c_int, [C.c_void_p, C.c_int64]),
    "pg_num_grids": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "pg_grid_info": (C.c_int, [C.c_void_p, C.c_int32] + [C.POINTER(C.c_int32)] * 6),
    "pg_recurrence_drift": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "pg_graph_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "pg_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.POINTER(Options)]),
    "pg_sweep_launch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pg_read_voltages": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int64]),
    "pg_read_voltages_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64]),
    "pg_read_inductor_currents": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int64]),
    "pg_update_mesh_values": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]),
    "pg_update_mesh_values_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pg_loss_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                  C.POINTER(C.c_double)]),
    "pg_loss_backward": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "pg_loss_backward_dev": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pg_loss_branch_gradients": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pg_loss_inductance_gradients": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pg_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "pg_reset_stats": (C.c_int, [C.c_void_p]),
    "pg_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "pg_read_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(KernelTimes)]),
}


def lib():
    """Load libpgrid.so (built in-tree by ``paper_1409_7166_amd.build``); fail loudly if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1409_7166_amd.build` "
                               "(the transient has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class _MeshHold:
    """Keeps the numpy buffers behind a MeshStruct alive."""
    struct: MeshStruct
    arrays: tuple


def mesh_struct(mesh) -> _MeshHold:
    """Marshal an object with the ``workloads.Mesh`` attributes into a ``pg_mesh``."""
    arrs = dict(gE=_f64(mesh.gE), gN=_f64(mesh.gN), C=_f64(mesh.C), via_node=_i32(mesh.via_node),
                via_g=_f64(mesh.via_g), via_L=_f64(mesh.via_L), pad_node=_i32(mesh.pad_node),
                pad_g=_f64(mesh.pad_g), pad_L=_f64(mesh.pad_L))
    nv, npd = int(arrs["via_node"].size), int(arrs["pad_node"].size)
    s = MeshStruct(int(mesh.nx), int(mesh.ny), int(mesh.nl), _dp(arrs["gE"]), _dp(arrs["gN"]), _dp(arrs["C"]),
                   nv, _ip(arrs["via_node"]), _dp(arrs["via_g"]),
                   _dp(arrs["via_L"]) if arrs["via_L"] is not None and arrs["via_L"].size else None,
                   npd, _ip(arrs["pad_node"]), _dp(arrs["pad_g"]),
                   _dp(arrs["pad_L"]) if arrs["pad_L"] is not None and arrs["pad_L"].size else None,
                   float(mesh.vdd))
    return _MeshHold(s, tuple(arrs.values()))


def _msgbuf():
    return C.create_string_buffer(512)


def validate_mesh(mesh):
    """Host-only check; returns (status, message)."""
    hold = mesh_struct(mesh)
    buf = _msgbuf()
    st = lib().pg_validate_mesh(C.byref(hold.struct), buf, 512)
    return st, buf.value.decode()


def _kinds(kind):
    k = np.asarray(kind)
    if k.dtype.kind in "US":
        k = np.frombuffer("".join(k.astype(str).ravel().tolist()).encode(), np.uint8)
    return np.ascontiguousarray(k, dtype=np.uint8)


def validate_netlist(n, p, frm, to, kind, value):
    """Host-only check of a branch list (kinds 'R', 'C', 'L', 'I'); returns (status, message)."""
    frm, to, value = _i32(frm), _i32(to), _f64(value)
    k = _kinds(kind)
    buf = _msgbuf()
    st = lib().pg_validate_netlist(int(n), int(p), int(frm.size), _ip(frm), _ip(to),
                                   k.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(value), buf, 512)
    return st, buf.value.decode()


@dataclass
class NetlistMesh:
    """The layered-mesh form of a netlist (the fields of a ``pg_mesh``)."""
    nx: int
    ny: int
    nl: int
    gE: np.ndarray
    gN: np.ndarray
    C: np.ndarray
    via_node: np.ndarray
    via_g: np.ndarray
    via_L: np.ndarray
    pad_node: np.ndarray
    pad_g: np.ndarray
    pad_L: np.ndarray
    vdd: float

    @property
    def n(self) -> int:
        return self.nl * self.ny * self.nx


def _netlist_args(n, p, source_v, frm, to, kind, value, dims):
    return (int(n), int(p), _f64(np.asarray(source_v, float).reshape(-1)), _i32(frm), _i32(to), _kinds(kind),
            _f64(value), None if dims is None else _i32(np.asarray(dims).reshape(3)))


@dataclass
class GraphShape:
    """Sizes of a general-netlist grid (pg_graph_info)."""
    n: int
    n_colors: int
    n_slots: int
    nnz: int
    n_inductors: int


def netlist_coloring(n, p, source_v, frm, to, kind, value):
    """Host-only: (color[n], slot[n], n_colors, n_slots) of a general netlist (pg_netlist_coloring)."""
    n, p, sv, frm, to, k, value, _ = _netlist_args(n, p, source_v, frm, to, kind, value, None)
    color, slot = np.zeros(n, np.int32), np.zeros(n, np.int32)
    nc, ns = C.c_int32(), C.c_int64()
    buf = _msgbuf()
    st = lib().pg_netlist_coloring(n, p, _dp(sv), int(frm.size), _ip(frm), _ip(to),
                                   k.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(value), _ip(color), _ip(slot),
                                   C.byref(nc), C.byref(ns), buf, 512)
    if st != 0:
        raise PgError(st, buf.value.decode())
    return color, slot, nc.value, ns.value


def netlist_to_mesh(n, p, source_v, frm, to, kind, value, dims):
    """Host-only: the mesh form of a netlist (pg_netlist_to_mesh); raises PGError if it has none."""
    n, p, sv, frm, to, k, value, dims = _netlist_args(n, p, source_v, frm, to, kind, value, dims)
    buf = _msgbuf()
    nv, npd = C.c_int32(), C.c_int32()
    kp = k.ctypes.data_as(C.POINTER(C.c_uint8))
    st = lib().pg_netlist_mesh_counts(n, p, _dp(sv), int(frm.size), _ip(frm), _ip(to), kp, _dp(value), _ip(dims),
                                      C.byref(nv), C.byref(npd), buf, 512)
    if st != 0:
        raise PgError(st, buf.value.decode())
    nx, ny, nl = (int(d) for d in dims)
    out = NetlistMesh(nx, ny, nl, np.zeros(nl * ny * (nx - 1)), np.zeros(nl * (ny - 1) * nx), np.zeros(nx * ny * nl),
                      np.zeros(nv.value, np.int32), np.zeros(nv.value), np.zeros(nv.value),
                      np.zeros(npd.value, np.int32), np.zeros(npd.value), np.zeros(npd.value), 0.0)
    vdd = C.c_double()
    st = lib().pg_netlist_to_mesh(n, p, _dp(sv), int(frm.size), _ip(frm), _ip(to), kp, _dp(value), _ip(dims),
                                  _dp(out.gE), _dp(out.gN), _dp(out.C), _ip(out.via_node), _dp(out.via_g),
                                  _dp(out.via_L), _ip(out.pad_node), _dp(out.pad_g), _dp(out.pad_L),
                                  C.byref(vdd), buf, 512)
    if st != 0:
        raise PgError(st, buf.value.decode())
    out.vdd = vdd.value
    out.gE = out.gE.reshape(nl, ny, nx - 1)
    out.gN = out.gN.reshape(nl, ny - 1, nx)
    out.C = out.C.reshape(nl, ny, nx)
    return out


def default_options(**kw) -> Options:
    o = Options()
    lib().pg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def validate_options(o: Options):
    buf = _msgbuf()
    st = lib().pg_validate_options(C.byref(o), buf, 512)
    return st, buf.value.decode()


class Context:
    """One pg_ctx on one GPU.  ``stream`` is a hipStream_t handle (int) or None."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        h = C.c_void_p()
        st = L.pg_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
        if st != 0:
            raise PgError(st, f"pg_create(device={device}) failed")
        self._h = h
        self.meshes = []

    # -- plumbing ------------------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise PgError(st, lib().pg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().pg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration -----------------------------------------------------------------------
    def set_options(self, **kw) -> Options:
        o = Options()
        self._check(lib().pg_get_options(self._h, C.byref(o)))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(lib().pg_set_options(self._h, C.byref(o)))
        return o

    def options(self) -> dict:
        o = Options()
        self._check(lib().pg_get_options(self._h, C.byref(o)))
        return {f: getattr(o, f) for f, _ in Options._fields_}

    def upload_mesh(self, mesh, n_scen: int = 1) -> int:
        hold = mesh_struct(mesh)
        gid = C.c_int32()
        self._check(lib().pg_upload_mesh(self._h, C.byref(hold.struct), int(n_scen), C.byref(gid)))
        self.meshes.append(mesh)
        return gid.value

    def upload_netlist(self, n, p, source_v, frm, to, kind, value, dims=None, n_scen: int = 1) -> int:
        """Upload a netlist (pg_upload_netlist): through its layered-mesh form when ``dims`` =
        (nx, ny, nl) is given, else as a general graph swept in colour order."""
        mesh = None if dims is None else netlist_to_mesh(n, p, source_v, frm, to, kind, value, dims)
        n, p, sv, frm, to, k, value, dims = _netlist_args(n, p, source_v, frm, to, kind, value, dims)
        gid = C.c_int32()
        self._check(lib().pg_upload_netlist(self._h, n, p, _dp(sv), int(frm.size), _ip(frm), _ip(to),
                                            k.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(value),
                                            _ip(dims) if dims is not None else None, int(n_scen), C.byref(gid)))
        self.meshes.append(mesh if mesh is not None else self.graph_info(gid.value))
        return gid.value

    def recurrence_drift(self, grid: int = 0, scen: int = 0) -> float:
        """KCL residual of the current state with the tracked inductor currents (three-level mode)."""
        d = C.c_double()
        self._check(lib().pg_recurrence_drift(self._h, grid, scen, C.byref(d)))
        return d.value

    def graph_info(self, grid: int) -> GraphShape:
        n, nc, ni = C.c_int32(), C.c_int32(), C.c_int32()
        ns, nnz = C.c_int64(), C.c_int64()
        self._check(lib().pg_graph_info(self._h, grid, C.byref(n), C.byref(nc), C.byref(ns), C.byref(nnz),
                                        C.byref(ni)))
        return GraphShape(n.value, nc.value, ns.value, nnz.value, ni.value)

    def sweep_launch_info(self) -> tuple:
        """(sweeps per mesh sweep launch, whether every fused launch stages its tiles once)."""
        spl, staged = C.c_int32(), C.c_int32()
        self._check(lib().pg_sweep_launch_info(self._h, C.byref(spl), C.byref(staged)))
        return spl.value, bool(staged.value)

    def _n_nodes(self, grid: int) -> int:
        m = self.meshes[grid]
        return int(m.n) if isinstance(m, GraphShape) else int(m.nx) * int(m.ny) * int(m.nl)

    def _n_branches(self, grid: int) -> int:
        m = self.meshes[grid]
        if isinstance(m, GraphShape):
            return int(m.n_inductors)
        return int(np.asarray(m.via_node).size + np.asarray(m.pad_node).size)

    def set_pulses(self, grid: int, scen: int, pulses):
        node, peak = _i32(pulses.node), _f64(pulses.peak)
        start, width = _f64(pulses.start), _f64(pulses.width)
        self._check(lib().pg_set_pulses(self._h, grid, scen, int(node.size), _ip(node), _dp(peak),
                                        _dp(start), _dp(width)))

    def set_pwl(self, grid: int, scen: int, node, offsets, t, i):
        node, offsets, t, i = _i32(node), _i32(offsets), _f64(t), _f64(i)
        self._check(lib().pg_set_pwl(self._h, grid, scen, int(node.size), _ip(node), _ip(offsets),
                                     _dp(t), _dp(i)))

    def set_state(self, grid: int, scen: int, v=None, i_l=None):
        v, i_l = _f64(v), _f64(i_l)
        self._check(lib().pg_set_state(self._h, grid, scen, _dp(v), _dp(i_l)))

    def reset(self):
        self._check(lib().pg_reset(self._h))

    def estimate_omega(self, grid: int = 0, dc: bool = False, iters: int = 512):
        """(rho_J, Young's omega) of the grid's step (or DC) matrix."""
        rho, w = C.c_double(), C.c_double()
        self._check(lib().pg_estimate_omega(self._h, grid, int(bool(dc)), int(iters), C.byref(rho), C.byref(w)))
        return rho.value, w.value

    def error_bound_factor(self, grid: int = 0, rel_tol: float = 1e-8) -> float:
        """||M^-1 D||_inf of the grid's step matrix: tol = err / kappa bounds a step's error by err."""
        k = C.c_double()
        self._check(lib().pg_error_bound_factor(self._h, grid, float(rel_tol), C.byref(k)))
        return k.value

    def error_bound_factor_noalloc(self, grid: int = 0, rel_tol: float = 1e-8) -> float:
        """error_bound_factor through the allocation-free entry point (fixed device scratch)."""
        k = C.c_double()
        self._check(lib().pg_error_bound_factor_noalloc(self._h, grid, float(rel_tol), C.byref(k)))
        return k.value

    def dc_operating_point(self, k: int = 0, omega: float = 0.0, tol: float = 1e-10, max_sweeps: int = 100000):
        """Set every state to the DC point with the sources at t = k h, and the clock to k."""
        self._check(lib().pg_dc_operating_point(self._h, int(k), float(omega), float(tol), int(max_sweeps)))

    # -- stepping --------------------------------------------------------------------------
    def step(self, nsteps: int = 1):
        self._check(lib().pg_step(self._h, int(nsteps)))

    def step_enqueue(self, nsteps: int = 1):
        """Queue nsteps steps on the context's stream without waiting (resident path; capturable)."""
        self._check(lib().pg_step_enqueue(self._h, int(nsteps)))

    def run_transient(self, nsteps: int, record_every: int = 1, grid: int = 0, scen: int = 0):
        n = self._n_nodes(grid)
        out = np.empty((nsteps // record_every, n))
        self._check(lib().pg_run_transient(self._h, int(nsteps), int(record_every), grid, scen,
                                           _dp(out) if out.size else None))
        return out

    def set_time_index(self, step: int):
        self._check(lib().pg_set_time(self._h, int(step)))

    def grid_info(self, grid: int = 0) -> dict:
        vals = [C.c_int32() for _ in range(6)]
        self._check(lib().pg_grid_info(self._h, grid, *[C.byref(v) for v in vals]))
        return dict(zip(("nx", "ny", "nl", "n_scen", "n_vias", "n_pads"), (v.value for v in vals)))

    def autotune(self, nsteps: int = 20, cache_path=None) -> dict:
        """Time candidate settings over `nsteps` steps from the current state and keep the fastest."""
        o = Options()
        self._check(lib().pg_autotune(self._h, int(nsteps), cache_path.encode() if cache_path else None,
                                      C.byref(o)))
        return {f: getattr(o, f) for f, _ in Options._fields_}

    def time_index(self) -> int:
        k = C.c_int64()
        self._check(lib().pg_get_time(self._h, C.byref(k)))
        return k.value

    # -- reads ---------------------------------------------------------------------------------
    def read_voltages(self, grid: int = 0, scen: int = 0) -> np.ndarray:
        n = self._n_nodes(grid)
        out = np.empty(n)
        self._check(lib().pg_read_voltages(self._h, grid, scen, _dp(out), n))
        return out

    def read_voltages_dev(self, grid: int, scen: int, tensor):
        """Copy into a float64 CUDA tensor (queued on the context stream)."""
        self._check(lib().pg_read_voltages_dev(self._h, grid, scen, C.c_void_p(tensor.data_ptr()),
                                               int(tensor.numel())))

    def read_inductor_currents(self, grid: int = 0, scen: int = 0) -> np.ndarray:
        nb = self._n_branches(grid)
        out = np.zeros(max(nb, 1))
        self._check(lib().pg_read_inductor_currents(self._h, grid, scen, _dp(out), nb))
        return out[:nb]

    # -- softplus voltage-drop loss and its adjoint ---------------------------------------------
    def update_mesh_values(self, grid: int, gE=None, gN=None, C=None):
        gE, gN, C = _f64(gE), _f64(gN), _f64(C)
        self._check(lib().pg_update_mesh_values(self._h, grid, _dp(gE), _dp(gN), _dp(C)))

    def update_mesh_values_dev(self, grid: int, gE=None, gN=None, C=None):
        """pg_update_mesh_values_dev: float64 CUDA tensors of the shapes of pg_mesh's gE, gN, C
        (None: unchanged), read on the context's stream."""
        info = self.grid_info(grid)
        nx, ny, nl = info["nx"], info["ny"], info["nl"]
        want = {"gE": nl * ny * (nx - 1), "gN": nl * (ny - 1) * nx, "C": nl * ny * nx}
        ptrs = []
        for name, t in (("gE", gE), ("gN", gN), ("C", C)):
            if t is None:
                ptrs.append(None)
                continue
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
            if t.numel() != want[name]:
                raise ValueError(f"{name} has {t.numel()} entries, the grid needs {want[name]}")
            ptrs.append(_VOIDP(t.data_ptr()))
        self._check(lib().pg_update_mesh_values_dev(self._h, grid, *ptrs))

    def loss_forward(self, grid: int, scen: int, nsteps: int, ckpt_every: int, margin: float) -> float:
        J = C.c_double()
        self._check(lib().pg_loss_forward(self._h, grid, scen, int(nsteps), int(ckpt_every), float(margin),
                                          C.byref(J)))
        return J.value

    def loss_backward(self, tol_adj: float, grid: int = 0):
        """Host arrays dJ/dC [nl,ny,nx], dJ/dgE [nl,ny,nx-1], dJ/dgN [nl,ny-1,nx]."""
        m = self.meshes[grid]
        nl, ny, nx = int(m.nl), int(m.ny), int(m.nx)
        dC, dE, dN = np.empty((nl, ny, nx)), np.empty((nl, ny, nx - 1)), np.empty((nl, ny - 1, nx))
        self._check(lib().pg_loss_backward(self._h, float(tol_adj), _dp(dC), _dp(dE), _dp(dN)))
        return dC, dE, dN

    def _branch_out(self, fn, grid):
        m = self.meshes[grid]
        nv, npd = np.asarray(m.via_node).size, np.asarray(m.pad_node).size
        dv, dp = np.zeros(max(1, nv)), np.zeros(max(1, npd))
        self._check(fn(self._h, _dp(dv), _dp(dp)))
        return dv[:nv], dp[:npd]

    def loss_branch_gradients(self, grid: int = 0):
        """(dJ/dvia_g [n_vias], dJ/dpad_g [n_pads]) of the last loss_backward."""
        return self._branch_out(lib().pg_loss_branch_gradients, grid)

    def loss_inductance_gradients(self, grid: int = 0):
        """(dJ/dvia_L [n_vias], dJ/dpad_L [n_pads]) of the last loss_backward (0 for resistive branches)."""
        return self._branch_out(lib().pg_loss_inductance_gradients, grid)

    def loss_backward_dev(self, tol_adj: float, dC, dE, dN):
        """Gradients into float64 device tensors (contiguous, shapes as in loss_backward)."""
        self._check(lib().pg_loss_backward_dev(self._h, float(tol_adj), C.c_void_p(dC.data_ptr()),
                                               C.c_void_p(dE.data_ptr()), C.c_void_p(dN.data_ptr())))

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().pg_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        self._check(lib().pg_reset_stats(self._h))

    def profile(self, every: int = 1):
        self._check(lib().pg_profile(self._h, int(every)))

    def kernel_times(self) -> dict:
        k = KernelTimes()
        self._check(lib().pg_read_kernel_times(self._h, C.byref(k)))
        return k.as_dict()
