"""GPU: the separate stage-update pass (Eqs. 2-8 with the RK4 stage combine) in both of
its work-group mappings, against the oracle's RK4 trajectory: tiles of 128 columns by 2
rows (nx a multiple of 128, ny even) and 256 consecutive columns (any other plane).
The grids run with the fused stage pass switched off, so every stage takes this pass."""
import numpy as np
import pytest

import oracle
from synthetic import random_unit_m
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

F, T = False, True
# (dims, periodic): two-row tiles with a ragged last z chunk; one plane per thread;
# two column tiles per row pair; wrapped x and y neighbours; odd ny and nx not a
# multiple of 128 (consecutive columns, rows split across work-groups)
CASES = [((128, 4, 3), (F, F, F)), ((128, 2, 1), (F, F, F)), ((256, 2, 2), (F, F, F)),
         ((128, 6, 2), (T, T, F)), ((128, 5, 2), (F, F, F)), ((96, 6, 3), (F, F, T))]


@pytest.mark.parametrize("dims,periodic", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_stage_update_mappings_match_oracle(dims, periodic, precision):
    nx, ny, nz = dims
    pb = oracle.Problem(nx, ny, nz, 4e-9, Ms=8e5, A=1.3e-11, Ku=3e3, alpha=0.3,
                        hext=(1.2e4, -3e3, 5e3), periodic=periodic)
    sim = mmag.Sim(nx, ny, nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=pb.Ku, alpha=pb.alpha, gamma=pb.gamma,
                   precision=precision, periodic=periodic, split_stage=True)
    assert sim.plan()["fused_stage"] == 0
    sim.set_hext(pb.hext)
    sim.set_m(random_unit_m(pb.shape, seed=nx + 7 * ny + 31 * nz))
    m0 = to_np(sim.get_m())
    dt, steps = 5e-14, 20
    sim.step(steps, dt)
    m = to_np(sim.get_m())
    ref = oracle.rk4(pb, m0, dt, steps)
    err = np.abs(m - ref).max()
    assert err <= (1e-11 if precision == "f64" else 2e-5), err
    sim.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_full_film_euler_step_sampled_against_oracle(precision):
    # The 512x512x16 film at full size in the default launch configuration (two-row
    # tiles): one explicit Euler step (the stage update's stage 0) at the 1024 seeded
    # observation cells against the oracle: its direct-sum demag field there, its
    # exchange and anisotropy fields, its LLG right-hand side, then the step and the
    # renormalisation the oracle's Euler integrator applies.
    import synthetic
    c = synthetic.LARGE
    pb = oracle.Problem(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha,
                        gamma=c.gamma, hext=tuple(c.hext))
    sim = mmag.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                   precision=precision)
    assert sim.plan()["fused_stage"] == 0
    sim.set_hext(c.hext)
    sim.set_m(random_unit_m(pb.shape, seed=103))
    m0 = to_np(sim.get_m()).reshape(3, -1)
    sim.step_euler(1, c.dt)
    m1 = to_np(sim.get_m()).reshape(3, -1)
    obs = synthetic.observation_cells(c.nx, c.ny, c.nz, 1024, seed=104)
    h = oracle.demag(pb, m0.reshape(pb.shape), obs) + \
        oracle.exchange(pb, m0.reshape(pb.shape)).reshape(3, -1)[:, obs] + \
        oracle.anisotropy(pb, m0.reshape(pb.shape)).reshape(3, -1)[:, obs] + \
        np.asarray(c.hext, dtype=np.float64).reshape(3, 1)
    n = len(obs)
    ps = oracle.Problem(n, 1, 1, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                        hext=tuple(c.hext))
    k = oracle.llg_rhs(ps, m0[:, obs].reshape(3, 1, 1, n), h.reshape(3, 1, 1, n)).reshape(3, n)
    v = m0[:, obs] + c.dt * k
    ref = v / np.sqrt((v * v).sum(axis=0))
    err = np.abs(m1[:, obs] - ref).max()
    print(f"full film Euler step {precision}: {err:.2e} over {n} cells")
    assert err <= (1e-12 if precision == "f64" else 2e-6), err
    sim.close()
