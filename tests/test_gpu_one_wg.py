"""The one-work-group demag evaluation (MM_ONE_WG: the whole padded volume of a
small grid transformed in LDS, Eq. 14 product, inverse) against the multi-pass
schedules and against the oracle's direct sum (Eqs. 12-14)."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import random_unit_m
from tests.gpu_util import rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}
# (dims, periodic, threads): 64x16, 16x12x4, 10x8x6, 20x14x6 (512 threads), periodic
# 15x12 (odd period: mirrored bins without a Nyquist bin)
CASES = [((32, 8, 1), (False, False, False), 0),
         ((8, 6, 2), (False, False, False), 0),
         ((5, 4, 3), (False, False, False), 0),
         ((10, 7, 3), (False, False, False), 512),
         ((15, 6, 1), (True, False, False), 0),
         ((6, 5, 4), (True, True, True), 0)]


def make(dims, precision, periodic=(False, False, False), **kw):
    nx, ny, nz = dims
    s = mmag.Sim(nx, ny, nz, 4e-9, Ms=8e5, A=1.3e-11, Ku=2e3, alpha=0.3, precision=precision,
                 periodic=periodic, images=1 if any(periodic) else 0, **kw)
    s.set_hext([1e4, -2e3, 3e3])
    return s


def problem(dims, periodic):
    return oracle.Problem(*dims, 4e-9, Ms=8e5, A=1.3e-11, Ku=2e3, alpha=0.3, hext=(1e4, -2e3, 3e3),
                          periodic=periodic, images=1 if any(periodic) else 0)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims,periodic,threads", CASES)
def test_one_wg_matches_multi_pass_and_oracle(dims, periodic, threads, precision):
    one = make(dims, precision, periodic, one_wg=True, threads=threads)
    multi = make(dims, precision, periodic, threads=threads)
    assert one.plan()["passes"] == 1 and multi.plan()["passes"] in (3, 5)
    m0 = random_unit_m((3, dims[2], dims[1], dims[0]), seed=sum(dims) + threads)
    one.set_m(m0)
    multi.set_m(m0)
    h1, hm = to_np(one.field("demag")), to_np(multi.field("demag"))
    assert rel_max(h1, hm) <= (1e-13 if precision == "f64" else 1e-6)
    pb = problem(dims, periodic)
    m = to_np(one.get_m())
    ref = oracle.heff_terms(pb, m)
    assert rel_max(h1, ref["demag"]) <= FIELD_TOL[precision]
    assert rel_max(to_np(one.field("eff")), ref["eff"]) <= FIELD_TOL[precision]
    e1, er = one.energy(), oracle.energy(pb, m)
    assert np.abs(e1 - er).max() <= (1e-10 if precision == "f64" else 1e-5) * np.abs(er).max()
    one.step(12, 1e-13)
    ref_m = oracle.rk4(pb, m, 1e-13, 12)
    assert np.abs(to_np(one.get_m()) - ref_m).max() <= (1e-11 if precision == "f64" else 2e-5)
    one.close()
    multi.close()


def test_one_wg_graph_replay_and_euler():
    dims = (32, 8, 1)
    outs = []
    for graph in (False, True):
        s = make(dims, "f32", one_wg=True, graph=graph)
        s.set_m(random_unit_m((3, 1, 8, 32), seed=4))
        s.step(19, 1e-13)
        s.step_euler(9, 1e-13)
        outs.append(to_np(s.get_m()))
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_one_wg_is_ignored_where_the_volume_does_not_fit():
    # the default schedule of this grid (the two-plane one: two cells thick) runs instead
    s = make((64, 48, 2), "f32", one_wg=True)
    d = make((64, 48, 2), "f32")
    assert s.plan()["passes"] == d.plan()["passes"] != 1
    assert s.plan()["two_plane"] == d.plan()["two_plane"]
    s.close()
    d.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_one_wg_adjoint_matches_oracle_adjoint(precision):
    nx, ny, nz = 6, 5, 2
    g = np.random.default_rng(5)
    ku = 500.0 + 50.0 * g.standard_normal((nz, ny, nx))
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.1, ku_map=ku, hext=(4e3, -1.5e3, 3e3))
    sim = mmag.Sim(nx, ny, nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=0.0, alpha=pb.alpha, gamma=pb.gamma,
                   precision=precision, one_wg=True)
    assert sim.plan()["passes"] == 1
    sim.set_hext(pb.hext)
    sim.set_ku_map(ku)
    sim.set_m(random_unit_m(pb.shape, 3))
    m_used = to_np(sim.get_m())
    w = g.standard_normal(pb.shape)
    dt, nsteps, ck = 1e-13, 12, 5
    ckpt = sim.rollout_ckpt(nsteps, dt, ck)
    dku, dm0 = sim.backward(nsteps, dt, ck, ckpt, torch.tensor(w, dtype=sim.dtype, device=sim.device))
    ref_ku, ref_m0 = oracle.rk4_adjoint(pb, m_used, dt, nsteps, w)
    tol = 1e-9 if precision == "f64" else 1e-4
    assert rel_max(to_np(dku), ref_ku) <= tol
    assert rel_max(to_np(dm0), ref_m0) <= tol
    sim.close()


def test_autotune_times_the_one_wg_schedule():
    # the small strip of 32x8x1 cells: the tuner times the one-work-group schedule
    # beside the multi-pass ones and keeps whichever is fastest
    s = make((32, 8, 1), "f32", autotune=True)
    p = s.plan()
    assert p["tuned"] == 1 and p["passes"] in (1, 3)
    s.set_m(random_unit_m((3, 1, 8, 32), seed=9))
    pb = problem((32, 8, 1), (False, False, False))
    assert rel_max(to_np(s.field("demag")), oracle.demag(pb, to_np(s.get_m()))) <= FIELD_TOL["f32"]
    s.close()
