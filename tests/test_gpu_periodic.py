"""Periodic boundaries (MM_PERIODIC_X/Y/Z, the alternative to zero padding named in
Sec. 2.3) on the GPU against the oracle's direct sum over the same image window,
and the uniformly magnetised periodic box against the union-prism closed form."""
import itertools

import numpy as np
import pytest

import oracle
from synthetic import random_unit_m
from tests.gpu_util import rel_max, to_np
from tests.test_oracle_periodic import apply, axis_windows, prism_tensor

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}

CASES = [
    # dims, periodic (x, y, z), images
    ((16, 12, 3), (True, True, False), 0),
    ((20, 15, 4), (True, True, True), 1),
    ((32, 8, 1), (True, False, False), 2),
    ((24, 10, 1), (False, True, False), 0),
    ((9, 7, 5), (False, False, True), 3),
    ((64, 64, 2), (True, True, False), 1),
    ((24, 32, 1), (False, True, False), 1),     # one cell thick, periodic y: whole-line y k-space
    ((32, 16, 4), (True, True, True), 0),       # every axis periodic, powers of two
]


def problem(dims, periodic, images, tensor="point", **kw):
    nx, ny, nz = dims
    return oracle.Problem(nx, ny, nz, 4e-9, Ms=8e5, A=1.3e-11, Ku=3e3, alpha=0.3,
                          hext=(1.2e4, -3e3, 5e3), periodic=periodic, images=images, tensor=tensor,
                          **kw)


def make_sim(pb, precision, **kw):
    s = mmag.Sim(pb.nx, pb.ny, pb.nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=pb.Ku, alpha=pb.alpha,
                 gamma=pb.gamma, precision=precision, periodic=pb.periodic, images=pb.images,
                 tensor=pb.tensor, **kw)
    s.set_hext(pb.hext)
    return s


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims,periodic,images", CASES)
def test_periodic_fields_match_oracle(dims, periodic, images, precision):
    pb = problem(dims, periodic, images)
    sim = make_sim(pb, precision)
    plan = sim.plan()
    for a, n, p in zip("xyz", dims, periodic):   # no padding along periodic axes
        if p:
            assert plan["p" + a] == n
    sim.set_m(random_unit_m(pb.shape, seed=sum(dims) + images))
    m = to_np(sim.get_m())
    ref = oracle.heff_terms(pb, m)
    for term in ("demag", "exch", "eff"):
        err = rel_max(to_np(sim.field(term)), ref[term])
        print(dims, periodic, images, precision, term, f"{err:.2e}")
        assert err <= FIELD_TOL[precision], (term, err)
    e_gpu, e_ref = sim.energy(), oracle.energy(pb, m)
    assert np.abs(e_gpu - e_ref).max() <= (1e-10 if precision == "f64" else 1e-5) * np.abs(e_ref).max()
    sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_periodic_newell_fields_match_oracle(precision):
    pb = problem((16, 16, 2), (True, True, False), 1, tensor="newell")
    sim = make_sim(pb, precision)
    sim.set_m(random_unit_m(pb.shape, seed=77))
    m = to_np(sim.get_m())
    err = rel_max(to_np(sim.field("demag")), oracle.demag(pb, m))
    assert err <= FIELD_TOL[precision], err
    sim.close()


@pytest.mark.parametrize("method", ["rk4", "euler"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_periodic_trajectory_matches_oracle(method, precision):
    pb = problem((12, 10, 3), (True, True, False), 1)
    sim = make_sim(pb, precision)
    sim.set_m(random_unit_m(pb.shape, seed=5))
    m0 = to_np(sim.get_m())
    dt, n = 1e-13, 12
    if method == "rk4":
        sim.step(n, dt)
        ref = oracle.rk4(pb, m0, dt, n)
    else:
        sim.step_euler(n, dt)
        ref = oracle.euler(pb, m0, dt, n)
    err = np.abs(to_np(sim.get_m()) - ref).max()
    assert err <= (1e-11 if precision == "f64" else 2e-5), err
    sim.close()


@pytest.mark.parametrize("dims,periodic,images", [((16, 12, 3), (True, True, False), 2),
                                                  ((15, 8, 4), (True, False, True), 1)])
def test_uniform_periodic_box_on_gpu_is_the_union_prism(dims, periodic, images):
    nx, ny, nz = dims
    sim = mmag.Sim(nx, ny, nz, 5e-9, Ms=8e5, precision="f64", periodic=periodic, images=images)
    u = np.array([0.6, -0.48, 0.64])
    sim.set_m(np.broadcast_to(u.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy())
    h = to_np(sim.field("demag"))
    worst = 0.0
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        ref = np.zeros(3)
        for (lx, hx, wx) in axis_windows(nx, periodic[0], images, i):
            for (ly, hy, wy) in axis_windows(ny, periodic[1], images, j):
                for (lz, hz, wz) in axis_windows(nz, periodic[2], images, k):
                    ref += wx * wy * wz * 8e5 * apply(prism_tensor((lx, ly, lz), (hx, hy, hz)), u)
        worst = max(worst, np.abs(h[:, k, j, i] - ref).max() / 8e5)
    assert worst < 1e-11, worst
    sim.close()


def test_periodic_film_full_size_sampled():
    # 512 x 512 x 16, periodic in x and y (FFT 512 x 512 x 32), FP32, default launch
    # configuration: demag and effective field at sampled cells against the oracle
    pb = oracle.Problem(512, 512, 16, 3e-9, Ms=8e5, A=1.3e-11, periodic=(True, True, False))
    sim = make_sim(pb, "f32")
    sim.set_m(random_unit_m(pb.shape, seed=11))
    m = to_np(sim.get_m())
    g = np.random.default_rng(12)
    obs = np.unique(np.concatenate([[0, 511, pb.N - 512, pb.N - 1], g.integers(0, pb.N, 48)]))
    err = rel_max(to_np(sim.field("demag")).reshape(3, -1)[:, obs], oracle.demag(pb, m, obs))
    ex = oracle.exchange(pb, m).reshape(3, -1)[:, obs]
    err_ex = rel_max(to_np(sim.field("exch")).reshape(3, -1)[:, obs], ex)
    print(f"periodic film: demag {err:.2e}, exchange {err_ex:.2e}")
    assert err <= FIELD_TOL["f32"] and err_ex <= FIELD_TOL["f32"]
    sim.step(5, 5e-14)
    mm = to_np(sim.get_m())
    assert np.abs(np.sqrt((mm * mm).sum(axis=0)) - 1).max() < 1e-6
    sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims,periodic", [((6, 5, 1), (True, True, False)),
                                           ((5, 4, 3), (True, False, True))])
def test_periodic_adjoint_matches_oracle_adjoint(dims, periodic, precision):
    # the reverse sweep wraps the exchange stencil of the covector like the forward step
    import torch
    g = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    ku = 500.0 + 50.0 * g.standard_normal((nz, ny, nx))
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.1, ku_map=ku, hext=(4e3, -1.5e3, 3e3),
                        periodic=periodic, images=1)
    sim = mmag.Sim(nx, ny, nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=0.0, alpha=pb.alpha, gamma=pb.gamma,
                   precision=precision, periodic=periodic, images=1)
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


def test_periodic_with_autotune_graph_and_schedule():
    # the autotuner keeps the period as the FFT length; graph replay and a
    # piecewise schedule run the same periodic step as plain stepping
    pb = problem((32, 24, 2), (True, False, False), 1)
    tuned = make_sim(pb, "f64", autotune=True)
    assert tuned.plan()["px"] == 32
    plain = make_sim(pb, "f64", graph=True)
    m0 = random_unit_m(pb.shape, seed=21)
    for s in (tuned, plain):
        s.set_m(m0)
        s.step(16, 1e-13)
    ref = oracle.rk4(pb, m0 / np.linalg.norm(m0, axis=0), 1e-13, 16)
    for s in (tuned, plain):
        assert np.abs(to_np(s.get_m()) - ref).max() <= 1e-11
    rows = plain.run_schedule([(8, pb.hext, (0.0, 0.0, 0.0), 0.3)], 1e-13, 4)
    _, m_ref = oracle.schedule(pb, ref, [(8, pb.hext, (0.0, 0.0, 0.0), 0.3)], 1e-13, 4)
    assert np.abs(to_np(plain.get_m()) - m_ref).max() <= 1e-11
    assert len(rows) == 2
    tuned.close()
    plain.close()


def test_periodic_z_of_one_cell():
    # a one-cell period along z: the cell is its own z neighbour (no exchange along
    # z) and every image of a source sits in the same plane stack
    pb = problem((6, 5, 1), (False, False, True), 2)
    sim = make_sim(pb, "f64")
    sim.set_m(random_unit_m(pb.shape, seed=31))
    m = to_np(sim.get_m())
    ref = oracle.heff_terms(pb, m)
    for term in ("demag", "exch"):
        assert rel_max(to_np(sim.field(term)), ref[term]) <= FIELD_TOL["f64"], term
    sim.close()
