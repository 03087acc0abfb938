"""GPU: the two-plane schedule of grids two cells thick (nz = 2).

There the z coupling of Eqs. 12-13 is split by z offset (observer minus source,
-1, 0 or +1) and each part convolved in x and y by Eq. 14, with no z transform.
Checked against the oracle (coefficient planes against numpy FFTs of the
oracle's tensor planes; fields, energies, RK4 trajectories and the adjoint
against the plain definitions), and against the five-pass schedule of the
runtime-radix passes, which transforms z.
"""
import numpy as np
import pytest

import oracle
from synthetic import mT_to_Apm, random_unit_m
from tests.gpu_util import problem, rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}


def make_sim(pb, precision, **kw):
    s = mmag.Sim(pb.nx, pb.ny, pb.nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=pb.Ku, alpha=pb.alpha,
                 gamma=pb.gamma, precision=precision, demag=pb.demag,
                 periodic=getattr(pb, "periodic", (False, False, False)), **kw)
    s.set_hext(pb.hext)
    return s


def plane_spectra(pb, Px, Py):
    """The 10 coefficient planes from numpy 2-D FFTs of the oracle's tensor
    planes at z offset 0 and +1 (wrapped padded layout), scaled 1/(Px Py),
    stored [kx][ky] over the first Py/2+1 ky."""
    tab = oracle.tensor_table(pb.nx, pb.ny, pb.nz)   # [6][2nz-1][2ny-1][2nx-1], offsets -(n-1)..n-1
    I = np.arange(-(pb.nx - 1), pb.nx) % Px
    J = np.arange(-(pb.ny - 1), pb.ny) % Py

    def fft_plane(c, d):
        w = np.zeros((Py, Px))
        w[np.ix_(J, I)] = tab[c][pb.nz - 1 + d]
        f = np.fft.fft2(w) / (Px * Py)
        return f[: Py // 2 + 1, : Px // 2 + 1].T            # [kx][ky]

    xx0, xx1 = fft_plane(0, 0), fft_plane(0, 1)
    xy0, xy1 = fft_plane(1, 0), fft_plane(1, 1)
    xz0, xz1 = fft_plane(2, 0), fft_plane(2, 1)
    yy0, yy1 = fft_plane(3, 0), fft_plane(3, 1)
    yz0, yz1 = fft_plane(4, 0), fft_plane(4, 1)
    zz0, zz1 = fft_plane(5, 0), fft_plane(5, 1)
    # the xz and yz planes vanish at offset 0 (odd in z) and are imaginary at +1
    # (odd in x resp. y); every other plane is real
    scale = max(np.abs(p).max() for p in (xx0, zz0))
    for p in (xz0, yz0):
        assert np.abs(p).max() <= 1e-14 * scale
    for p in (xx0, xx1, xy0, xy1, yy0, yy1, zz0, zz1):
        assert np.abs(p.imag).max() <= 1e-13 * scale
    assert np.abs(xz1.real).max() <= 1e-13 * scale and np.abs(yz1.real).max() <= 1e-13 * scale
    return np.array([xx0.real, xx1.real, xy0.real, xy1.real, xz1.imag, yy0.real, yy1.real,
                     yz1.imag, zz0.real, zz1.real])


@pytest.mark.parametrize("dims,kw", [((64, 48, 2), {}), ((20, 16, 2), {}), ((33, 47, 2), {"pow2_pad": True})])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_coefficient_planes_match_fft_of_oracle_tensor(dims, kw, precision):
    pb = problem(*dims, cell=5e-9)
    sim = make_sim(pb, precision, **kw)
    p = sim.plan()
    assert p["two_plane"] == 1 and p["passes"] == 3
    spec = to_np(sim.kernel_spectrum())
    ref = plane_spectra(pb, p["px"], p["py"])
    assert spec.shape == ref.shape
    assert p["kernel_imag_ratio"] <= 1e-12
    tol = 1e-12 if precision == "f64" else 1e-6
    assert rel_max(spec, ref) <= tol
    sim.close()


# (dims, options, periodic): specialised lengths pruned (power of two, mixed
# radix 96, 160), whole lines along a periodic y axis, and one column in x
CASES = [((64, 48, 2), {}, (False, False, False)),
         ((33, 47, 2), {"pow2_pad": True}, (False, False, False)),
         ((37, 80, 2), {"fast_pad": True}, (False, False, False)),
         ((1, 40, 2), {"fast_pad": True}, (False, False, False)),
         ((24, 32, 2), {}, (False, True, False)),
         ((16, 16, 2), {}, (True, True, False))]


@pytest.mark.parametrize("dims,kw,periodic", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_plane_fields_and_energies_match_oracle(dims, kw, periodic, precision):
    hext = mT_to_Apm([9.0, -4.0, 6.0])
    nx, ny, nz = dims
    pb = oracle.Problem(nx, ny, nz, 4e-9, Ms=8e5, A=1.3e-11, Ku=2.0e4, alpha=0.5,
                        hext=tuple(hext), periodic=periodic)
    sim = make_sim(pb, precision, **kw)
    p = sim.plan()
    assert p["two_plane"] == 1, p
    sim.set_m(random_unit_m(pb.shape, seed=nx + 3 * ny))
    m = to_np(sim.get_m())
    ref = oracle.heff_terms(pb, m)
    for term in ("demag", "eff"):
        err = rel_max(to_np(sim.field(term)), ref[term])
        print(dims, kw, periodic, precision, term, f"{err:.2e}")
        assert err <= FIELD_TOL[precision], (term, err)
    e_gpu, e_ref = sim.energy(), oracle.energy(pb, m)
    assert np.abs(e_gpu - e_ref).max() <= (1e-10 if precision == "f64" else 1e-5) * np.abs(e_ref).max()
    sim.close()


@pytest.mark.parametrize("dims", [(64, 48, 2), (96, 112, 2)])
def test_two_plane_matches_five_passes(dims):
    # the runtime-radix passes keep the five-pass schedule (z transformed): FP64
    # fields of both schedules agree to rounding
    pb = problem(*dims, cell=3e-9, Ku=1.0e4)
    m0 = random_unit_m(pb.shape, seed=11)
    out = []
    for generic in (False, True):
        sim = make_sim(pb, "f64", generic_fft=generic)
        assert sim.plan()["two_plane"] == (0 if generic else 1)
        sim.set_m(m0)
        out.append(to_np(sim.field("demag")))
        sim.close()
    assert rel_max(out[0], out[1]) <= 1e-13


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_plane_trajectory_matches_oracle(precision):
    pb = problem(20, 16, 2, cell=5e-9, Ku=500.0, alpha=0.5, hext=mT_to_Apm([3.0, 8.0, -5.0]))
    sim = make_sim(pb, precision)
    assert sim.plan()["two_plane"] == 1
    sim.set_m(random_unit_m(pb.shape, seed=5))
    m0 = to_np(sim.get_m())
    dt, n = 1e-13, 200
    sim.step(n, dt)
    ref = oracle.rk4(pb, m0, dt, n)
    err = np.abs(to_np(sim.get_m()) - ref).max()
    print(precision, f"{err:.2e}")
    assert err <= (1e-9 if precision == "f64" else 1e-4)
    sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_plane_adjoint_matches_oracle_adjoint(precision):
    import torch
    g = np.random.default_rng(12)
    nx, ny, nz = 16, 8, 2
    ku = 500.0 + 50.0 * g.standard_normal((nz, ny, nx))
    hext = mT_to_Apm([6.0, -2.0, 4.0])
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.1, ku_map=ku, hext=tuple(hext))
    sim = mmag.Sim(nx, ny, nz, 5e-9, Ms=pb.Ms, A=pb.A, Ku=0.0, alpha=pb.alpha, gamma=pb.gamma,
                   precision=precision)
    assert sim.plan()["two_plane"] == 1
    sim.set_hext(hext)
    sim.set_ku_map(ku)
    sim.set_m(random_unit_m(pb.shape, 4))
    m_used = to_np(sim.get_m())
    w = g.standard_normal(pb.shape)
    dt, nsteps, ck = 1e-13, 10, 4
    ckpt = sim.rollout_ckpt(nsteps, dt, ck)
    lam = torch.tensor(w, dtype=sim.dtype, device=sim.device)
    dku, dm0 = sim.backward(nsteps, dt, ck, ckpt, lam)
    ref_ku, ref_m0 = oracle.rk4_adjoint(pb, m_used, dt, nsteps, w)
    tol = 1e-9 if precision == "f64" else 1e-4
    assert rel_max(to_np(dku), ref_ku) <= tol
    assert rel_max(to_np(dm0), ref_m0) <= tol
    sim.close()


def test_batch_of_two_plane_grids_matches_single_runs_and_oracle():
    # a batch mixing one- and two-cell-thick grids under the size-class passes: the
    # two-plane grids run the batched two-plane pass
    grids = [(33, 47, 2), (40, 32, 1), (64, 64, 2), (17, 90, 2), (50, 50, 1)]
    hext = np.array([mT_to_Apm([5.0 * i, -3.0, 2.0 + i]) for i in range(len(grids))])
    b = mmag.BatchSim(grids, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5, hext=hext, precision="f32",
                      pow2_pad=True)
    assert b.info()["size_classes"] == 1
    ms = [random_unit_m((3, nz, ny, nx), seed=20 + i) for i, (nx, ny, nz) in enumerate(grids)]
    b.set_m(ms)
    m_used = [to_np(x) for x in b.get_m()]
    h = [to_np(x) for x in b.field("eff")]
    for i, (nx, ny, nz) in enumerate(grids):
        pb = oracle.Problem(nx, ny, nz, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5, hext=tuple(hext[i]))
        ref = oracle.heff_terms(pb, m_used[i])["eff"]
        assert rel_max(h[i], ref) <= 1e-5, (grids[i], rel_max(h[i], ref))
    dt, n = 1e-13, 20
    b.step(n, dt)
    got = [to_np(x) for x in b.get_m()]
    for i, (nx, ny, nz) in enumerate(grids):
        s = mmag.Sim(nx, ny, nz, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5, precision="f32",
                     pow2_pad=True)
        s.set_hext(hext[i])
        s.set_m(ms[i])
        s.step(n, dt)
        assert s.plan()["two_plane"] == (1 if nz == 2 else 0)
        assert np.abs(to_np(s.get_m()) - got[i]).max() <= 1e-6
        s.close()
    b.close()


def test_small_size_class_is_padded_into_the_next_and_stays_exact():
    # one 32x40 grid beside forty 100x100 grids: its x class (64 points) holds under
    # 1/32 of the cells, so it runs in the 256-point class; the field is unchanged
    grids = [(32, 40, 2)] + [(100, 100, 1)] * 40
    b = mmag.BatchSim(grids, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5, precision="f64", pow2_pad=True)
    assert b.info()["size_classes"] == 1
    p0, p1 = b.grid_plan(0), b.grid_plan(1)
    assert (p1["px"], p1["py"]) == (256, 256)
    assert (p0["px"], p0["py"]) == (256, 256) and p0["two_plane"] == 1 and p0["passes"] == 3
    with pytest.raises(mmag.MMError):
        b.grid_plan(len(grids))
    b.set_m([random_unit_m((3, nz, ny, nx), seed=i) for i, (nx, ny, nz) in enumerate(grids)])
    m0 = to_np(b.get_m()[0])
    h0 = to_np(b.field("demag")[0])
    pb = oracle.Problem(32, 40, 2, 5e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.5)
    assert rel_max(h0, oracle.demag(pb, m0)) <= FIELD_TOL["f64"]
    b.close()
