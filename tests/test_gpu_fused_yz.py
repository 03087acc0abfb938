"""The fused y-z pass (three passes per field evaluation) against the five
separate passes and against the oracle's direct sum (Eqs. 12-14)."""
import numpy as np
import pytest

import oracle
from synthetic import random_unit_m
from tests.gpu_util import rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}
GRIDS = [(256, 64, 4), (20, 15, 3), (64, 48, 5), (100, 30, 2), (7, 9, 6)]


def sim(dims, precision, **kw):
    nx, ny, nz = dims
    return mmag.Sim(nx, ny, nz, 4e-9, Ms=8e5, A=1.3e-11, Ku=2e3, alpha=0.3, precision=precision, **kw)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims", GRIDS)
def test_fused_yz_matches_five_passes_and_oracle(dims, precision):
    fused, five = sim(dims, precision, fused_yz=True), sim(dims, precision)
    assert fused.plan()["passes"] == 3 and five.plan()["passes"] == 5
    m0 = random_unit_m((3, dims[2], dims[1], dims[0]), seed=sum(dims))
    fused.set_m(m0)
    five.set_m(m0)
    hf, h5 = to_np(fused.field("demag")), to_np(five.field("demag"))
    assert rel_max(hf, h5) <= (1e-13 if precision == "f64" else 1e-6)
    if dims[0] * dims[1] * dims[2] <= 20000:
        pb = oracle.Problem(*dims, 4e-9, Ms=8e5, A=1.3e-11, Ku=2e3, alpha=0.3)
        assert rel_max(hf, oracle.demag(pb, to_np(fused.get_m()))) <= FIELD_TOL[precision]
    fused.step(10, 1e-13)
    five.step(10, 1e-13)
    assert np.abs(to_np(fused.get_m()) - to_np(five.get_m())).max() <= (1e-13 if precision == "f64" else 1e-6)
    fused.close()
    five.close()


def test_autotune_times_fused_and_five_pass_schedules():
    s = sim((256, 64, 4), "f32", autotune=True)
    p = s.plan()
    assert p["tuned"] == 1 and p["passes"] in (3, 5)
    s.close()
