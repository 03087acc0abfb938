"""Edge cases of the stepping entry points: zero steps, and graph replay across
changes of the applied field, damping, time step and anisotropy map (each change
must be seen by the next replay exactly as by plain launches)."""
import numpy as np
import pytest

from synthetic import random_unit_m
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_zero_steps_leave_m_unchanged(graph, precision):
    sim = mmag.Sim(13, 7, 3, 5e-9, Ku=400.0, alpha=0.2, precision=precision, graph=graph)
    sim.set_m(random_unit_m((3, 3, 7, 13), seed=2))
    m0 = to_np(sim.get_m())
    sim.step(0, 1e-13)
    sim.step_euler(0, 1e-13)
    assert np.array_equal(to_np(sim.get_m()), m0)
    sim.step(1, 1e-13)
    assert not np.array_equal(to_np(sim.get_m()), m0)
    sim.close()


def test_batch_zero_steps_leave_m_unchanged():
    b = mmag.BatchSim([(20, 9, 1), (11, 13, 2)], 5e-9, precision="f32", graph=True)
    b.set_m([random_unit_m((3, 1, 9, 20), seed=3), random_unit_m((3, 2, 13, 11), seed=4)])
    m0 = to_np(b.get_m_flat())
    b.step(0, 1e-13)
    assert np.array_equal(to_np(b.get_m_flat()), m0)
    b.step(1, 1e-13)
    assert not np.array_equal(to_np(b.get_m_flat()), m0)
    b.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_graph_replay_follows_parameter_changes(precision):
    nx, ny, nz = 24, 10, 2
    m0 = random_unit_m((3, nz, ny, nx), seed=7)
    ku = 300.0 + 40.0 * np.random.default_rng(8).standard_normal((nz, ny, nx))
    outs = []
    for graph in (False, True):
        sim = mmag.Sim(nx, ny, nz, 4e-9, Ku=500.0, alpha=0.3, precision=precision, graph=graph)
        sim.set_hext([1e4, 0.0, 0.0])
        sim.set_m(m0)
        sim.step(9, 1e-13)                 # one replay of 8 steps + 1 plain step
        sim.set_hext([0.0, -2e4, 5e3])
        sim.step(9, 1e-13)
        sim.set_alpha(0.05)
        sim.step(9, 1e-13)
        sim.step(9, 2e-13)                 # another time step
        sim.set_ku_map(ku)
        sim.step(9, 2e-13)
        sim.set_ku_map(None)               # back to the uniform Ku
        sim.step_euler(9, 1e-13)
        sim.step(9, 2e-13)
        outs.append(to_np(sim.get_m()))
        sim.close()
    assert np.array_equal(outs[0], outs[1])
