"""Shapes, counts and determinism of the seeded workloads."""
import numpy as np
import pytest

from workloads import config0, config2, config3b, config4, small_multilayer


def test_config0_counts():
    w = config0()
    m = w.meshes[0]
    assert m.n == 1024 and m.gE.size + m.gN.size == 1984
    assert m.pad_node.size == 16 and w.pulses[0][0].count == 1024
    assert np.all((m.gE >= 0.5) & (m.gE <= 2.0)) and np.all((m.C >= 0.5e-12) & (m.C <= 2e-12))
    assert w.h == 10e-12 and w.steps == 100


def test_deterministic():
    a, b = config0(), config0()
    assert np.array_equal(a.meshes[0].gE, b.meshes[0].gE)
    assert np.array_equal(a.pulses[0][0].start, b.pulses[0][0].start)


def test_multilayer_recipe_small():
    w = small_multilayer(side=128, seed=1)
    m = w.meshes[0]
    assert m.nl == 3 and m.via_node.size == 2 * 32 * 32 and m.pad_node.size == 4
    assert np.all(m.pad_node >= 2 * 128 * 128)
    assert np.all(m.C[1:] == 0) and np.all(m.C[0] > 0)
    assert w.pulses[0][0].count == round(0.3 * 128 * 128)
    assert np.all(w.pulses[0][0].node < 128 * 128)


@pytest.mark.slow
def test_config2_and_config4_counts():
    w = config2()
    m = w.meshes[0]
    assert m.n == 524288 and m.gE.size + m.gN.size == 1046528
    assert m.via_node.size == 16384 and m.pad_node.size == 64
    assert np.all((m.via_L >= 1e-12) & (m.via_L <= 10e-12))
    w4 = config4()
    m4 = w4.meshes[0]
    assert m4.n == 1048576 and m4.gE.size + m4.gN.size == 2095104 and m4.pad_node.size == 256


def test_config3b_sides():
    w = config3b()
    assert len(w.meshes) == 64
    assert set(w.extra["sides"]) <= {64, 128, 256, 512}
