"""The allocation-free entry point pg_error_bound_factor_noalloc against pg_error_bound_factor.

Both compute kappa = ||M^-1 D||_inf of a grid's step matrix with the same kernels; the variant
keeps the grid's saved state in the library's fixed device scratch instead of a buffer allocated
per call.  Two calls in a row (a 3-layer grid, then a smaller single-layer one, so the second
call finds the first one's contents in the scratch) must each give the allocating entry point's
result and leave the state bit for bit as it was; the smaller kappa is also checked against the
oracle's direct computation.  Sizes beyond the scratch and a context whose coefficients are not
built yet are refused with an error."""
import numpy as np
import pytest

import paper_1409_7166_amd as pg
from helpers import compressed, gpu_context, say
from oracle import BESystem, error_bound_factor, mesh_to_circuit
from workloads import small_multilayer, small_rc

pytestmark = pytest.mark.gpu


def _stepped(w, prec, steps):
    ctx = gpu_context(w, precision=prec, tol=1e-10, omega=1.5)
    ctx.step(steps)
    return ctx


@pytest.mark.parametrize("prec", [pg.PG_PREC_FP64, pg.PG_PREC_FP32_REFINE])
def test_noalloc_matches_the_allocating_entry_point_on_two_calls(prec):
    wa = small_multilayer(side=96, seed=5, nl=3, pad_every=16, steps=20)
    wb = small_rc(40, 33, seed=6, steps=20)
    wb.pulses[0][0] = compressed(wb.pulses[0][0], start=0.02, width=0.5)
    say(f"[gpu] noalloc kappa prec={prec}: 3x96x96 then 1x40x33")
    with _stepped(wa, prec, 6) as ca, _stepped(wb, prec, 4) as cb:
        va, vb = ca.read_voltages(), cb.read_voltages()
        assert np.max(1.0 - vb) > 1e-6  # the saved state is not the trivial one
        ka_na = ca.error_bound_factor_noalloc(0, rel_tol=1e-10)
        assert np.array_equal(ca.read_voltages(), va)
        kb_na = cb.error_bound_factor_noalloc(0, rel_tol=1e-10)   # smaller grid, same scratch
        assert np.array_equal(cb.read_voltages(), vb)
        ka = ca.error_bound_factor(0, rel_tol=1e-10)
        kb = cb.error_bound_factor(0, rel_tol=1e-10)
        assert np.array_equal(ca.read_voltages(), va) and np.array_equal(cb.read_voltages(), vb)
        # the transient goes on from the restored state as from the untouched one
        ca.step(2)
        va2 = ca.read_voltages()
    with _stepped(wa, prec, 8) as twin:
        va_twin = twin.read_voltages()
    circ, _ = mesh_to_circuit(wb.meshes[0], None)
    kb_ref = error_bound_factor(BESystem(circ, wb.h).M)
    say(f"  kappa 3x96x96: noalloc {ka_na:.12g} alloc {ka:.12g}; 1x40x33: noalloc {kb_na:.12g} "
        f"alloc {kb:.12g} oracle {kb_ref:.12g}")
    assert ka_na == pytest.approx(ka, rel=1e-12)
    assert kb_na == pytest.approx(kb, rel=1e-12)
    assert kb_na == pytest.approx(kb_ref, rel=1e-7)
    assert np.max(np.abs(va2 - va_twin)) <= 1e-12


def test_noalloc_refuses_unbuilt_coefficients_and_oversized_grids():
    w = small_rc(24, 20, seed=7, steps=5)
    with gpu_context(w, precision=pg.PG_PREC_FP64) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.error_bound_factor_noalloc(0)
        assert ei.value.name == "PG_ERR_STATE"
        ctx.step(1)
        assert ctx.error_bound_factor_noalloc(0, rel_tol=1e-9) > 1.0
    big = small_rc(2052, 2048, seed=8, steps=1)  # 2052 * 2048 = 4,202,496 slots > 2^22
    say("[gpu] noalloc refuses a 2052x2048 grid")
    with gpu_context(big, precision=pg.PG_PREC_FP32_REFINE) as ctx:
        with pytest.raises(pg.PgError) as ei:
            ctx.error_bound_factor_noalloc(0)
        assert ei.value.name == "PG_ERR_INVALID_ARG"
        assert "at most 4194304" in str(ei.value)
