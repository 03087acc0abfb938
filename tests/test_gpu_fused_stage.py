"""GPU: the fused stage pass of small grids (x inverse, stage update and x forward of the
stage output in one launch; the y / z passes run between its launches) against the
separate passes (MM_SPLIT_STAGE) and against the oracle, on one-cell-thick grids, grids
two cells thick (two-plane schedule) and thicker 3-D grids."""
import numpy as np
import pytest

import oracle
from synthetic import mT_to_Apm, random_unit_m
from tests.gpu_util import rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")


def make(dims, precision, Ku=500.0, alpha=0.5, hext=(4.0, -7.0, 2.0), **kw):
    nx, ny, nz = dims
    s = mmag.Sim(nx, ny, nz, 5e-9, Ms=8e5, A=1.3e-11, Ku=Ku, alpha=alpha, precision=precision, **kw)
    s.set_hext(mT_to_Apm(list(hext)))
    return s


# (dims, options): the strip of the small workload, the 128x128 film, power-of-two
# and mixed-radix padding, rows not a multiple of the block, one column; two cells
# thick (the two-plane y pass between the fused launches); the mid-size film, a
# cube and ragged 3-D grids (y forward, z k-space, y inverse between them), with
# one, two and four row pairs per work-group
GRIDS = [((32, 8, 1), {}), ((128, 128, 1), {}), ((100, 37, 1), {"pow2_pad": True}),
         ((45, 61, 1), {"fast_pad": True}), ((17, 24, 1), {"pow2_pad": True}), ((64, 9, 1), {"pow2_pad": True}),
         ((64, 48, 2), {}), ((33, 47, 2), {"pow2_pad": True}), ((256, 64, 4), {}), ((32, 32, 32), {}),
         ((40, 21, 3), {"pow2_pad": True}), ((45, 30, 5), {"fast_pad": True}), ((60, 64, 20), {"pow2_pad": True})]


@pytest.mark.parametrize("dims,kw", GRIDS)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_stage_matches_separate_passes(dims, kw, precision):
    fused, split = make(dims, precision, **kw), make(dims, precision, split_stage=True, **kw)
    assert fused.plan()["fused_stage"] == 1, fused.plan()
    assert split.plan()["fused_stage"] == 0
    m0 = random_unit_m((3, dims[2], dims[1], dims[0]), seed=sum(dims))
    for s in (fused, split):
        s.set_m(m0)
        s.step(13, 1e-13)
    a, b = to_np(fused.get_m()), to_np(split.get_m())
    assert np.abs(a - b).max() <= (1e-13 if precision == "f64" else 2e-6)
    fused.close()
    split.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_stage_graph_replay_and_readouts_in_between(precision):
    # graph replay (8-step groups plus a remainder) equals eager launches bitwise; a
    # field readout between step calls overwrites the spectrum buffer, which the next
    # call's prologue forms again
    dims = (96, 48, 1)
    eager, graph = make(dims, precision), make(dims, precision, graph=True)
    m0 = random_unit_m((3, 1, 48, 96), seed=3)
    for s in (eager, graph):
        s.set_m(m0)
        s.step(19, 1e-13)
        s.field("eff")
        s.step(5, 1e-13)
    assert np.array_equal(to_np(eager.get_m()), to_np(graph.get_m()))
    split = make(dims, precision, split_stage=True)
    split.set_m(m0)
    split.step(24, 1e-13)
    assert np.abs(to_np(eager.get_m()) - to_np(split.get_m())).max() <= (1e-13 if precision == "f64" else 2e-6)
    for s in (eager, graph, split):
        s.close()


@pytest.mark.parametrize("dims", [(40, 24, 1), (20, 12, 3)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_stage_trajectory_matches_oracle(precision, dims):
    hext = mT_to_Apm([3.0, 8.0, -5.0])
    pb = oracle.Problem(*dims, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5, hext=tuple(hext))
    sim = make(dims, precision, pow2_pad=True, hext=(3.0, 8.0, -5.0))
    assert sim.plan()["fused_stage"] == 1
    sim.set_m(random_unit_m(pb.shape, seed=9))
    m0 = to_np(sim.get_m())
    dt, n = 1e-13, 300
    sim.step(n, dt)
    err = np.abs(to_np(sim.get_m()) - oracle.rk4(pb, m0, dt, n)).max()
    print(precision, f"{err:.2e}")
    assert err <= (1e-9 if precision == "f64" else 1e-4)
    sim.close()


@pytest.mark.parametrize("dims", [(32, 16, 1), (16, 8, 3)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_stage_rollout_adjoint_matches_oracle_adjoint(precision, dims):
    # the rollout (checkpointed forward) runs the fused stages, and so does the
    # reverse sweep's recompute of each segment (storing every stage's field)
    import torch
    g = np.random.default_rng(31)
    nx, ny, nz = dims
    ku = 500.0 + 50.0 * g.standard_normal((nz, ny, nx))
    hext = mT_to_Apm([6.0, -2.0, 4.0])
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.1, ku_map=ku, hext=tuple(hext))
    sim = mmag.Sim(nx, ny, nz, 5e-9, Ms=pb.Ms, A=pb.A, Ku=0.0, alpha=pb.alpha, gamma=pb.gamma,
                   precision=precision)
    assert sim.plan()["fused_stage"] == 1
    sim.set_hext(hext)
    sim.set_ku_map(ku)
    sim.set_m(random_unit_m(pb.shape, 4))
    m_used = to_np(sim.get_m())
    w = g.standard_normal(pb.shape)
    dt, nsteps, ck = 1e-13, 12, 5
    ckpt = sim.rollout_ckpt(nsteps, dt, ck)
    m_end = to_np(sim.get_m())
    assert np.abs(m_end - oracle.rk4(pb, m_used, dt, nsteps)).max() <= (1e-11 if precision == "f64" else 1e-5)
    lam = torch.tensor(w, dtype=sim.dtype, device=sim.device)
    dku, dm0 = sim.backward(nsteps, dt, ck, ckpt, lam)
    ref_ku, ref_m0 = oracle.rk4_adjoint(pb, m_used, dt, nsteps, w)
    tol = 1e-9 if precision == "f64" else 1e-4
    assert rel_max(to_np(dku), ref_ku) <= tol
    assert rel_max(to_np(dm0), ref_m0) <= tol
    sim.close()


def test_fused_stage_is_not_taken_where_it_does_not_apply():
    # periodic axes, runtime-radix passes, beyond 2^20 cells: the separate passes
    assert make((32, 32, 1), "f32", periodic=(True, False, False)).plan()["fused_stage"] == 0
    assert make((32, 32, 8), "f32", periodic=(False, False, True)).plan()["fused_stage"] == 0
    assert make((128, 128, 128), "f32").plan()["fused_stage"] == 0
    assert make((32, 32, 1), "f32", generic_fft=True).plan()["fused_stage"] == 0
    assert make((30, 30, 1), "f32").plan()["fused_stage"] == 0   # 60 points: no specialised pass


@pytest.mark.parametrize("dims,kw", [((32, 8, 1), {}), ((16, 16, 16), {}), ((40, 21, 3), {"pow2_pad": True}),
                                     ((64, 48, 2), {})])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_euler_matches_separate_passes(dims, kw, precision):
    # the explicit Euler step (stage 0) through the fused pass: odd counts (the result
    # copied back), an RK4 call in between, graph replay of 8-step groups plus a
    # remainder bitwise equal to eager launches, and the separate passes to rounding
    m0 = random_unit_m((3, dims[2], dims[1], dims[0]), seed=sum(dims) + 1)
    runs = {}
    for name, opts in (("eager", {}), ("graph", {"graph": True}), ("split", {"split_stage": True})):
        s = make(dims, precision, alpha=1.0, **kw, **opts)
        assert s.plan()["fused_stage"] == (0 if name == "split" else 1)
        s.set_m(m0)
        s.step_euler(21, 1e-13)
        s.step(3, 1e-13)
        s.step_euler(19, 1e-13)
        runs[name] = to_np(s.get_m())
        s.close()
    assert np.array_equal(runs["eager"], runs["graph"])
    assert np.abs(runs["eager"] - runs["split"]).max() <= (1e-13 if precision == "f64" else 2e-6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_euler_matches_oracle(precision):
    # standard-problem-#3-like material on a fused 3-D plan against the oracle's Euler
    Ms = 1.0e6
    Ku = 4e-7 * np.pi * Ms * 1.0e5 / 2
    dims = (10, 7, 3)
    pb = oracle.Problem(*dims, 4e-9, Ms=Ms, A=1e-11, Ku=Ku, alpha=1.0)
    sim = mmag.Sim(*dims, 4e-9, Ms=Ms, A=1e-11, Ku=Ku, alpha=1.0, precision=precision, pow2_pad=True)
    assert sim.plan()["fused_stage"] == 1
    sim.set_m(random_unit_m(pb.shape, seed=31))
    m_used = to_np(sim.get_m())
    sim.step_euler(25, 2e-14)
    err = np.abs(to_np(sim.get_m()) - oracle.euler(pb, m_used, 2e-14, 25)).max()
    assert err <= (1e-11 if precision == "f64" else 2e-5), err
    sim.close()


@pytest.mark.parametrize("dims", [(24, 16, 1), (24, 16, 2), (20, 12, 3)])
@pytest.mark.parametrize("method", ["euler", "rk4"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_schedule_with_ramps_matches_separate_passes(dims, method, precision):
    # a time-dependent protocol (field ramps, a damping switch, a constant piece) on
    # fused plans: the applied field changes every step inside the fused launches
    pieces = [(7, (1e4, 0.0, 0.0), (2e4, 5e3, 0.0), 0.5), (9, (2e4, 5e3, 0.0), (2e4, 5e3, 0.0), 0.02),
              (6, (0.0, 1e4, 0.0), (-1e4, 0.0, 3e3), 0.3)]
    dt = 2e-14 if method == "euler" else 1e-13
    m0 = random_unit_m((3, dims[2], dims[1], dims[0]), seed=77)
    out = {}
    for split in (False, True):
        s = make(dims, precision, pow2_pad=True, split_stage=split)
        assert s.plan()["fused_stage"] == (0 if split else 1)
        s.set_m(m0)
        rows = to_np(s.run_schedule(pieces, dt, 4, method=method))
        out[split] = (rows, to_np(s.get_m()))
        s.close()
    tol = 1e-13 if precision == "f64" else 2e-6
    assert np.abs(out[False][0] - out[True][0]).max() <= tol
    assert np.abs(out[False][1] - out[True][1]).max() <= tol
