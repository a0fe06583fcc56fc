"""CPU tests of the C ABI: the library loads, exports every declared symbol, and the
host-only validation follows the topological assumptions of Sec. III-B."""
import os
import re

import numpy as np
import pytest

import paper_1409_7166_amd as pg
from paper_1409_7166_amd import pgrid as binding
from workloads import Mesh, config0, small_multilayer, small_rlc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pgrid.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pg.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
        assert n in binding.EXPORTS, f"binding lacks {n}"
    assert L.pg_abi_version() == 1
    assert L.pg_status_name(-3) == b"PG_ERR_NOT_SPD"


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pg.PgError) as ei:
        pg.Context(0)
    assert ei.value.name == "PG_ERR_DEVICE"


def test_valid_workloads_pass_validation():
    for w in (config0(), small_multilayer(side=64, seed=2), small_rlc(side=32, seed=3)):
        assert pg.validate_mesh(w.meshes[0]) == (0, "")


def _copy(m, **kw):
    d = {k: getattr(m, k) for k in ("nx", "ny", "nl", "gE", "gN", "C", "via_node", "via_g", "via_L",
                                    "pad_node", "pad_g", "pad_L", "vdd")}
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    d.update(kw)
    return Mesh(**d)


def test_mesh_validation_errors():
    m = config0().meshes[0]
    gE = m.gE.copy(); gE[0, 3, 4] = np.nan
    st, msg = pg.validate_mesh(_copy(m, gE=gE))
    assert st == -1 and "gE" in msg
    C = m.C.copy(); C[0, 0, 0] = -1e-12
    assert pg.validate_mesh(_copy(m, C=C))[0] == -1
    assert pg.validate_mesh(_copy(m, pad_node=m.pad_node + 5000))[0] == -1
    assert pg.validate_mesh(_copy(m, nl=5, C=np.zeros((5, 32, 32))))[0] == -8


def test_floating_island_is_not_spd():
    """Cut one corner node off (zero conductances), give it no pad and no capacitor."""
    m = config0().meshes[0]
    gE, gN, C = m.gE.copy(), m.gN.copy(), m.C.copy()
    y, x = 31, 31
    gE[0, y, x - 1] = 0.0
    gN[0, y - 1, x] = 0.0
    C[0, y, x] = 0.0
    st, msg = pg.validate_mesh(_copy(m, gE=gE, gN=gN, C=C))
    assert st == -3 and "component" in msg
    # a capacitor anchors it again (C/h on the diagonal)
    C[0, y, x] = 1e-12
    assert pg.validate_mesh(_copy(m, gE=gE, gN=gN, C=C))[0] == 0


def test_netlist_assumptions():
    # two trivial nodes, one supply: R(0-2), R(0-1), C(1-gnd): fine
    ok = pg.validate_netlist(2, 1, [0, 0, 1], [2, 1, -1], "RRC", [1.0, 2.0, 1e-12])
    assert ok[0] == 0, ok
    # node 1 touched only by a current source: violates assumption 2
    st, msg = pg.validate_netlist(2, 1, [0, 1], [2, -1], "RI", [1.0, 0.0])
    assert st == -2 and "current sources" in msg
    # node 1 only has a capacitor to ground: no branch to another non-ground node
    assert pg.validate_netlist(2, 1, [0, 1], [2, -1], "RC", [1.0, 1e-12])[0] == -2
    # sub-circuit {2,3} joined to nothing but itself (Fig. 1 split) with no anchor: singular
    st, msg = pg.validate_netlist(4, 1, [0, 1, 2], [4, 0, 3], "RRR", [1.0, 1.0, 1.0])
    assert st == -3
    # the same sub-circuit with an inductor to the supply is definite (h L term)
    assert pg.validate_netlist(4, 1, [0, 1, 2, 3], [4, 0, 3, 4], "RRRL", [1, 1, 1, 1e-12])[0] == 0
    assert pg.validate_netlist(2, 1, [0, 0], [2, 7], "RR", [1.0, 1.0])[0] == -1
    assert pg.validate_netlist(2, 1, [0, 0], [2, 1], "RX", [1.0, 1.0])[0] == -1
    assert pg.validate_netlist(2, 1, [0, 0], [2, 1], "RR", [1.0, -1.0])[0] == -1


def test_options_validation():
    o = pg.default_options()
    assert pg.validate_options(o)[0] == 0
    assert (o.h, o.tol, o.omega, o.check_every) == (10e-12, 1e-6, 1.0, 8)
    for k, v in (("omega", 2.0), ("omega", 0.0), ("h", 0.0), ("h", float("nan")), ("tol", -1.0),
                 ("max_sweeps", 0), ("check_every", 0), ("precision", 5), ("ordering", 3),
                 ("tile_rows", 12), ("lookahead", 9), ("recurrence", 2), ("sweeps_per_launch", 3),
                 ("sweeps_per_launch", 5), ("predictor", 3)):
        bad = pg.default_options(**{k: v})
        st, msg = pg.validate_options(bad)
        assert st == -1, (k, v)
    # four sweeps per launch in either precision (tile groups without the kernel sweep once per launch)
    assert pg.validate_options(pg.default_options(sweeps_per_launch=4))[0] == 0
    assert pg.validate_options(pg.default_options(sweeps_per_launch=4, precision=pg.PG_PREC_FP32_REFINE))[0] == 0
    # the predictor runs with plain launches only
    st, msg = pg.validate_options(pg.default_options(predictor=1, graphs=1))
    assert st == -8 and "plain launches" in msg
    assert pg.validate_options(pg.default_options(predictor=1))[0] == 0
    assert pg.validate_options(pg.default_options(predictor=2))[0] == 0
    assert pg.validate_options(pg.default_options(predictor=2, graphs=1))[0] == -8
    # the three-level recurrence runs with plain launches only
    st, msg = pg.validate_options(pg.default_options(recurrence=pg.PG_REC_THREE_LEVEL, graphs=1))
    assert st == -8 and "plain launches" in msg
    assert pg.validate_options(pg.default_options(recurrence=pg.PG_REC_THREE_LEVEL))[0] == 0
