"""Error paths that need the device: invalid magnetisation is refused at
mm_set_m (zero-length or non-finite cells, counted by the normalising kernel),
and a run driven unstable reports MM_ENONFINITE from its reductions instead of
returning numbers; the per-kernel event profile times the launches it is asked to."""
import numpy as np
import pytest

from synthetic import random_unit_m

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")


@pytest.mark.parametrize("bad", ["zero", "nan", "inf"])
def test_set_m_rejects_invalid_cells_and_step_then_refuses(bad):
    sim = mmag.Sim(12, 7, 2, 4e-9, precision="f32")
    m = random_unit_m((3, 2, 7, 12), seed=81)
    if bad == "zero":
        m[:, 1, 3, 5] = 0.0
    else:
        m[1, 0, 6, 11] = np.nan if bad == "nan" else np.inf
    with pytest.raises(mmag.MMError) as e:
        sim.set_m(m)
    assert e.value.status == -1 and "non-finite" in str(e.value)
    with pytest.raises(mmag.MMError) as e:
        sim.step(1, 1e-13)
    assert e.value.status == -4          # MM_ESTATE: no valid m
    sim.set_m(random_unit_m((3, 2, 7, 12), seed=82))   # a valid m restores the handle
    sim.step(2, 1e-13)
    assert np.isfinite(sim.mean_m()).all()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_unstable_run_reports_nonfinite(precision):
    # A finite but absurd applied field (1e300 A/m; beyond FP32's range once reduced)
    # makes the products of the RK4 stages overflow: Inf - Inf gives NaN in m, and
    # the reductions report it instead of returning numbers.
    sim = mmag.Sim(8, 8, 1, 5e-9, precision=precision)
    sim.set_m(random_unit_m((3, 1, 8, 8), seed=83))
    sim.set_hext([1e300, -5e299, 2e299])
    sim.step(3, 1e-6)
    m = sim.get_m().cpu().numpy()
    assert not np.isfinite(m).all()
    for call in (sim.mean_m, sim.energy):
        with pytest.raises(mmag.MMError) as e:
            call()
        assert e.value.status == -6      # MM_ENONFINITE


def test_profile_sampling_counts_launches():
    # one launch in `every` of the profiled kernel is bracketed by events
    sim = mmag.Sim(64, 32, 4, 5e-9, Ms=8e5, A=1.3e-11, Ku=0.0, alpha=0.5, precision="f32")
    sim.set_m(random_unit_m((3, 4, 32, 64), seed=4))
    sim.step(2, 1e-13)
    sim.profile_begin("kspace")
    sim.step(6, 1e-13)
    ms_all, n_all = sim.profile_end()
    assert n_all == 24 and ms_all > 0            # four field evaluations per RK4 step
    sim.profile_begin("kspace", every=5)
    sim.step(6, 1e-13)
    ms_s, n_s = sim.profile_end()
    assert n_s == 5 and ms_s > 0                  # launches 0, 5, 10, 15, 20 of 24
    assert 0.2 < (ms_s / n_s) / (ms_all / n_all) < 5
    with pytest.raises(mmag.MMError):
        sim.profile_begin("llg", every=0)
    sim.close()
