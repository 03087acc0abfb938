"""Batched form: many uneven grids advanced by one launch per pass, against the
same grids run one at a time and against the oracle."""
import numpy as np
import pytest

import oracle
from synthetic import BATCH_TEMPLATE, batch_samples, mT_to_Apm, random_unit_m
from tests.gpu_util import rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

C = BATCH_TEMPLATE
MIXED = [(33, 47, 1), (32, 32, 2), (64, 40, 1), (37, 128, 2), (128, 128, 1), (5, 3, 2),
         (1, 1, 1), (45, 32, 2), (97, 61, 1), (70, 3, 2)]


def fields_for(n, seed=0):
    g = np.random.default_rng(seed)
    return mT_to_Apm(g.uniform(-40, 40, size=(n, 3)))


def run_single(grid, hext, m0, precision, nsteps, pow2=False, generic=None, fast=False):
    nx, ny, nz = grid
    sim = mmag.Sim(nx, ny, nz, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                   precision=precision,
                   generic_fft=(not (pow2 or fast)) if generic is None else generic,
                   threads=256, pow2_pad=pow2, fast_pad=fast)
    sim.set_hext(hext)
    sim.set_m(m0)
    sim.step(nsteps, C.dt)
    return to_np(sim.get_m())


FAST_MIXED = [g for g in MIXED if min(g[0], g[1]) >= 8]   # power-of-two padding >= 16


@pytest.mark.parametrize("pad", ["7-smooth", "pow2", "fast"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_single_grid_runs(precision, pad):
    # runtime-radix passes on 7-smooth padding, or size classes of the specialised
    # passes on power-of-two or specialised-set padding: each grid as if run alone
    pow2, fast = pad == "pow2", pad == "fast"
    grids = FAST_MIXED if (pow2 or fast) else MIXED
    hext = fields_for(len(grids))
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=100 + i) for i, g in enumerate(grids)]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision=precision, pow2_pad=pow2, fast_pad=fast)
    assert b.info()["size_classes"] == int(pow2 or fast)
    b.set_m(m0)
    b.step(20, C.dt)
    got = [to_np(x) for x in b.get_m()]
    worst = 0.0
    for i, g in enumerate(grids):
        ref = run_single(g, hext[i], m0[i], precision, 20, pow2=pow2, fast=fast)
        worst = max(worst, float(np.abs(got[i] - ref).max()))
    print(f"batch vs single-grid runs ({precision}, {pad}): max |dm| = {worst:.3e}")
    assert worst <= (1e-13 if precision == "f64" else 1e-6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_oracle(precision):
    grids = [(6, 5, 1), (7, 4, 2), (9, 3, 1), (4, 4, 3)]
    hext = fields_for(len(grids), seed=3)
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=200 + i) for i, g in enumerate(grids)]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision=precision)
    b.set_m(m0)
    m_used = [to_np(x) for x in b.get_m()]
    b.step(15, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for i, g in enumerate(grids):
        pb = oracle.Problem(g[0], g[1], g[2], C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha,
                            gamma=C.gamma, hext=tuple(hext[i]))
        ref = oracle.rk4(pb, m_used[i], C.dt, 15)
        err = np.abs(got[i] - ref).max()
        assert err <= (1e-11 if precision == "f64" else 1e-5), (g, err)


def test_batch_graph_replay_matches_eager():
    hext = fields_for(len(MIXED), seed=5)
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=300 + i) for i, g in enumerate(MIXED)]
    outs = []
    for graph in (False, True):
        b = mmag.BatchSim(MIXED, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                          hext=hext, precision="f32", graph=graph)
        b.set_m(m0)
        b.step(19, C.dt)
        outs.append(to_np(b.get_m_flat()))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("pow2", [False, True])
def test_full_batched_workload_512_grids(pow2):
    # 512 grids, nx, ny uniform in [32, 128], nz in {1, 2}, fields in a 50 mT ball.
    samples = batch_samples(512, seed=0)
    grids = [(s.nx, s.ny, s.nz) for s in samples]
    hext = np.array([s.hext for s in samples])
    m0 = [random_unit_m((3, s.nz, s.ny, s.nx), seed=s.seed) for s in samples]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision="f32", graph=True, pow2_pad=pow2)
    b.set_m(m0)
    b.step(10, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for x in got:
        assert np.isfinite(x).all()
        assert np.abs(np.sqrt((x * x).sum(axis=0)) - 1).max() < 1e-6
    # the smallest, the largest and a few others against single-grid runs
    sizes = [g[0] * g[1] * g[2] for g in grids]
    pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 1, 100, 311, 511]))
    for i in pick:
        ref = run_single(grids[i], hext[i], m0[i], "f32", 10, pow2=pow2)
        assert np.abs(got[i] - ref).max() <= 1e-6, (i, grids[i])


def test_batch_with_newell_tensor_matches_single_grid_runs():
    grids = FAST_MIXED[:4]
    hext = fields_for(len(grids), seed=9)
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=400 + i) for i, g in enumerate(grids)]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision="f64", pow2_pad=True, tensor="newell")
    b.set_m(m0)
    b.step(10, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for i, g in enumerate(grids):
        nx, ny, nz = g
        sim = mmag.Sim(nx, ny, nz, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                       precision="f64", threads=256, pow2_pad=True, tensor="newell")
        sim.set_hext(hext[i])
        sim.set_m(m0[i])
        sim.step(10, C.dt)
        assert np.abs(got[i] - to_np(sim.get_m())).max() <= 1e-13


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_with_per_grid_materials_matches_single_grid_runs(precision):
    # Each grid its own Ms, A, Ku, alpha and gamma (MM_PER_GRID_MATERIAL).
    grids = MIXED[:6]
    n = len(grids)
    g = np.random.default_rng(17)
    Ms = g.uniform(6e5, 1.2e6, n)
    A = g.uniform(0.8e-11, 1.5e-11, n)
    Ku = g.uniform(0, 2e4, n)
    alpha = g.uniform(0.05, 0.8, n)
    gamma = np.full(n, 2.211e5) * g.uniform(0.9, 1.1, n)
    hext = fields_for(n, seed=11)
    m0 = [random_unit_m((3, gr[2], gr[1], gr[0]), seed=500 + i) for i, gr in enumerate(grids)]
    b = mmag.BatchSim(grids, C.cell, Ms=Ms, A=A, Ku=Ku, alpha=alpha, gamma=gamma, hext=hext,
                      precision=precision)
    b.set_m(m0)
    b.step(15, C.dt)
    b.step(5, 0.5 * C.dt)            # a second dt refreshes every grid's step factor
    got = [to_np(x) for x in b.get_m()]
    for i, (nx, ny, nz) in enumerate(grids):
        sim = mmag.Sim(nx, ny, nz, C.cell, Ms=Ms[i], A=A[i], Ku=Ku[i], alpha=alpha[i], gamma=gamma[i],
                       precision=precision, generic_fft=True, threads=256)
        sim.set_hext(hext[i])
        sim.set_m(m0[i])
        sim.step(15, C.dt)
        sim.step(5, 0.5 * C.dt)
        err = np.abs(got[i] - to_np(sim.get_m())).max()
        assert err <= (1e-13 if precision == "f64" else 1e-6), (i, err)



@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_autotuned_batch_matches_single_grid_runs_on_its_layout(precision):
    # MM_AUTOTUNE times the layouts and keeps one; the result is each grid run
    # alone with that layout's padding and pass family.
    grids = FAST_MIXED
    hext = fields_for(len(grids), seed=21)
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=600 + i) for i, g in enumerate(grids)]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision=precision, autotune=True)
    info = b.info()
    print(f"autotuned batch ({precision}): {info}")
    assert info["tuned"] == 1 and 2 <= info["candidates"] <= 4
    assert info["tuned_demag_ms"] > 0 and info["n"] == len(grids) and info["cells"] == b.cells
    assert not (info["size_classes"] and not (info["pow2_pad"] or info["fast_pad"]))
    b.set_m(m0)
    b.step(20, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for i, g in enumerate(grids):
        ref = run_single(g, hext[i], m0[i], precision, 20, pow2=bool(info["pow2_pad"]),
                         generic=not info["size_classes"], fast=bool(info["fast_pad"]))
        err = np.abs(got[i] - ref).max()
        assert err <= (1e-13 if precision == "f64" else 1e-6), (g, err)


def test_autotuned_batch_of_tiny_grids_keeps_a_buildable_layout():
    # grids whose power-of-two padding has no size-class pass: two candidates at most
    grids = [(5, 3, 2), (1, 1, 1), (70, 3, 2)]
    b = mmag.BatchSim(grids, C.cell, precision="f32", autotune=True)
    info = b.info()
    assert info["tuned"] == 1 and info["size_classes"] == 0 and info["candidates"] <= 2
    plain = mmag.BatchSim(grids, C.cell, precision="f32")
    assert plain.info()["tuned"] == 0 and plain.info()["pow2_pad"] == 0
