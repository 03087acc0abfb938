"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's formulas: each compares it with a
closed form, an invariant, an independent brute-force evaluation (surface
charge quadrature, finite differences of the energy) or a number printed in
the paper (tests/golden/paper_constants.json).
"""
import json
import os

import numpy as np
import pytest

import oracle
from synthetic import mT_to_Apm, random_unit_m

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
MU0 = 4e-7 * np.pi
XX, XY, XZ, YY, YZ, ZZ = range(6)


def full(k6):
    """6-vector (xx,xy,xz,yy,yz,zz) -> symmetric 3x3."""
    return np.array([[k6[XX], k6[XY], k6[XZ]], [k6[XY], k6[YY], k6[YZ]], [k6[XZ], k6[YZ], k6[ZZ]]])


# ----------------------------------------------------------------- tensor (Eqs. 10-11)
def test_tensor_origin_is_minus_third():
    # Each of the eight corner terms of Eq. 10 at the origin is -pi/6, so K(0) = -I/3.
    k = full(oracle.tensor_point(0, 0, 0))
    assert np.allclose(k, -np.eye(3) / 3.0, rtol=0, atol=2e-16 * 8)


def test_tensor_traceless_off_origin():
    # Outside the source cube the point field solves Laplace's equation: trace 0.
    g = np.random.default_rng(1)
    for _ in range(300):
        d = g.integers(-40, 41, size=3)
        if not d.any():
            continue
        k = oracle.tensor_point(*d)
        assert abs(k[XX] + k[YY] + k[ZZ]) < 1e-14


@pytest.mark.parametrize("dims,P", [((5, 4, 3), (10, 8, 6)), ((7, 3, 2), (14, 6, 4)), ((4, 4, 4), (7, 7, 7))])
def test_tensor_spectrum_trace_is_minus_one(dims, P):
    # Trace -1 at the origin and 0 elsewhere: the padded spectra (numpy FFT of the
    # wrapped table) satisfy Kxx + Kyy + Kzz = -1 at every frequency.
    nx, ny, nz = dims
    Px, Py, Pz = P
    tab = oracle.tensor_table(nx, ny, nz)
    I, J, K = (np.arange(-(n - 1), n) % q for n, q in zip(dims, P))
    tr = 0
    for c in (0, 3, 5):
        w = np.zeros((Pz, Py, Px))
        w[np.ix_(K, J, I)] = tab[c]
        tr = tr + np.fft.fftn(w)
    assert np.abs(tr + 1).max() < 1e-14


def test_tensor_parities_and_permutations():
    g = np.random.default_rng(2)
    for _ in range(200):
        I, J, K = (int(v) for v in g.integers(-25, 26, size=3))
        k = oracle.tensor_point(I, J, K)
        # even under d -> -d
        assert np.allclose(oracle.tensor_point(-I, -J, -K), k, rtol=1e-9, atol=2e-15)
        # reflections: xy odd in x and y, xz odd in x and z, yz odd in y and z
        kx = oracle.tensor_point(-I, J, K)
        ky = oracle.tensor_point(I, -J, K)
        kz = oracle.tensor_point(I, J, -K)
        sgn_x = np.array([1, -1, -1, 1, 1, 1])
        sgn_y = np.array([1, -1, 1, 1, -1, 1])
        sgn_z = np.array([1, 1, -1, 1, -1, 1])
        assert np.allclose(kx, sgn_x * k, rtol=1e-9, atol=2e-15)
        assert np.allclose(ky, sgn_y * k, rtol=1e-9, atol=2e-15)
        assert np.allclose(kz, sgn_z * k, rtol=1e-9, atol=2e-15)
        # relabelling axes permutes components (the "other components by permutation")
        assert np.isclose(oracle.tensor_point(J, I, K)[XX], k[YY], rtol=1e-9, atol=2e-15)
        assert np.isclose(oracle.tensor_point(K, J, I)[XX], k[ZZ], rtol=1e-9, atol=2e-15)
        assert np.isclose(oracle.tensor_point(I, K, J)[XY], k[XZ], rtol=1e-9, atol=2e-15)
        assert np.isclose(oracle.tensor_point(K, J, I)[XY], k[YZ], rtol=1e-9, atol=2e-15)


def test_tensor_independent_of_axis_zero_planes():
    for d in [(3, 0, 2), (0, 4, 1), (5, 2, 0), (0, 0, 3)]:
        k = oracle.tensor_point(*d)
        if d[0] == 0 or d[1] == 0:
            assert abs(k[XY]) < 2e-15
        if d[0] == 0 or d[2] == 0:
            assert abs(k[XZ]) < 2e-15
        if d[1] == 0 or d[2] == 0:
            assert abs(k[YZ]) < 2e-15


def dipole(d):
    d = np.asarray(d, dtype=float)
    r = np.sqrt(d @ d)
    return (3 * np.outer(d, d) - r * r * np.eye(3)) / (4 * np.pi * r ** 5)


def test_tensor_dipole_far_field():
    # Far from the source cube the field is that of a point dipole of moment M*delta^3;
    # the correction is O(1/|d|^2) relative.
    errs = []
    for s in (1, 2, 4):
        d = np.array([20, 13, 7]) * s
        k = full(oracle.tensor_point(*d))
        dp = dipole(d)
        errs.append(np.abs(k - dp).max() / np.abs(dp).max())
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * x, 0.5 * w       # on [-1/2, 1/2]


def surface_charge_field(d, axis, panels=6, order=12):
    """Field at the origin of a unit cube centred at d, magnetised along `axis`
    with unit M: H(p) = 1/(4 pi) sum over the two charged faces of
    int sigma (p - r') / |p - r'|^3 dA, by composite Gauss-Legendre quadrature."""
    x, w = _gauss(order)
    edges = np.linspace(-0.5, 0.5, panels + 1)
    pts, wts = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        pts.append(0.5 * (a + b) + (b - a) * x)
        wts.append((b - a) * w)
    u = np.concatenate(pts)
    wu = np.concatenate(wts)
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu)
    H = np.zeros(3)
    others = [a for a in range(3) if a != axis]
    for sigma, off in ((+1.0, +0.5), (-1.0, -0.5)):
        r = np.zeros((3,) + U.shape)
        r[axis] = d[axis] + off
        r[others[0]] = d[others[0]] + U
        r[others[1]] = d[others[1]] + V
        sep = -r                                 # p - r' with p = 0
        dist3 = np.sqrt((sep ** 2).sum(axis=0)) ** 3
        for a in range(3):
            H[a] += (sigma * W * sep[a] / dist3).sum()
    return H / (4 * np.pi)


@pytest.mark.parametrize("d", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (2, -1, 1),
                               (-3, 2, 5), (1, 2, 3)])
def test_tensor_matches_surface_charge_quadrature(d):
    # Independent brute force: the tensor column K[:, a] is the field at the observer
    # point of a cube uniformly magnetised along a (Sec. 2.3; Nakatani's point field).
    k = full(oracle.tensor_point(*d))
    for a in range(3):
        h = surface_charge_field(np.array(d, dtype=float), a)
        assert np.allclose(k[:, a], h, rtol=0, atol=2e-9), (d, a, k[:, a], h)


# ---------------------------------------------------------------- demag (Eqs. 12-13)
def test_single_cell_demag_is_minus_third():
    pb = oracle.Problem(1, 1, 1, 5e-9, Ms=8e5)
    m = np.array([0.6, 0.0, 0.8]).reshape(3, 1, 1, 1)
    h = oracle.demag(pb, m)
    assert np.allclose(h.reshape(3), -8e5 * np.array([0.6, 0.0, 0.8]) / 3, rtol=1e-14)


def test_uniform_cube_average_is_minus_third():
    # Cubic symmetry + trace -1: the cell-averaged demag tensor of an n^3 cube is -I/3.
    n = 4
    pb = oracle.Problem(n, n, n, 2e-9, Ms=1.0)
    for a in range(3):
        m = np.zeros(pb.shape)
        m[a] = 1.0
        h = oracle.demag(pb, m)
        avg = h.reshape(3, -1).mean(axis=1)
        expect = np.zeros(3)
        expect[a] = -1.0 / 3.0
        assert np.allclose(avg, expect, rtol=0, atol=1e-14)


def test_uniform_box_trace_and_ordering():
    # At every cell the three diagonal responses sum to -Ms (interior point of the body);
    # a 6x3x2 box has N_xx < N_yy < N_zz (smallest along the long axis).
    pb = oracle.Problem(6, 3, 2, 1e-9, Ms=1.0)
    diag = []
    for a in range(3):
        m = np.zeros(pb.shape)
        m[a] = 1.0
        diag.append(oracle.demag(pb, m)[a])
    tr = diag[0] + diag[1] + diag[2]
    assert np.allclose(tr, -1.0, rtol=0, atol=1e-14)
    nxx, nyy, nzz = (-d.mean() for d in diag)
    assert nxx < nyy < nzz
    assert abs(nxx + nyy + nzz - 1.0) < 1e-14


def test_thin_film_normal_factor():
    # A wide one-cell-thick film is close to the infinite-plate limit N_zz -> 1.
    pb = oracle.Problem(48, 48, 1, 1e-9, Ms=1.0)
    m = np.zeros(pb.shape)
    m[2] = 1.0
    nzz = -oracle.demag(pb, m)[2].mean()
    assert 0.9 < nzz < 1.0


def test_demag_sampled_observers_match_full():
    pb = oracle.Problem(7, 5, 3, 3e-9, Ms=8e5)
    m = random_unit_m(pb.shape, 3)
    h = oracle.demag(pb, m).reshape(3, -1)
    obs = np.array([0, 4, 17, 33, 104, 7 * 5 * 3 - 1])
    hs = oracle.demag(pb, m, obs)
    assert np.array_equal(hs, h[:, obs])


# --------------------------------------------------------------- exchange (Eqs. 5-7)
def test_exchange_zero_for_uniform():
    pb = oracle.Problem(5, 4, 3, 3e-9)
    m = np.zeros(pb.shape)
    m[0], m[1], m[2] = 0.48, -0.6, 0.64
    assert np.all(oracle.exchange(pb, m) == 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_exchange_linear_and_quadratic_profiles(axis):
    # Linear profile: zero inside, +-slope at the two end faces (Eq. 7's one-sided
    # difference).  Quadratic profile u = q^2: constant 2 inside.
    n = (6, 5, 4)
    pb = oracle.Problem(*n, cell=2e-9, Ms=8e5, A=1.3e-11)
    pref = 2 * pb.A / (MU0 * pb.Ms * pb.cell ** 2)
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    q = (x, y, z)[axis].astype(float)
    L = n[axis]
    for comp in range(3):
        m = np.zeros(pb.shape)
        m[comp] = 0.3 + 0.1 * q
        h = oracle.exchange(pb, m)[comp] / pref
        expect = np.where(q == 0, 0.1, np.where(q == L - 1, -0.1, 0.0))
        assert np.allclose(h, expect, rtol=0, atol=1e-14)
        m[comp] = q * q
        h = oracle.exchange(pb, m)[comp] / pref
        inner = (q > 0) & (q < L - 1)
        assert np.allclose(h[inner], 2.0, rtol=0, atol=1e-12)
        # boundary: Eq. 7, the missing neighbour equals the boundary cell
        assert np.allclose(h[q == 0], 1.0, rtol=0, atol=1e-12)
        lo = (L - 2) ** 2 - (L - 1) ** 2
        assert np.allclose(h[q == L - 1], lo, rtol=0, atol=1e-12)


def test_exchange_operator_symmetric_negative():
    pb = oracle.Problem(5, 4, 3, 3e-9)
    g = np.random.default_rng(4)
    u = g.standard_normal(pb.shape)
    v = g.standard_normal(pb.shape)
    Lu, Lv = oracle.exchange(pb, u), oracle.exchange(pb, v)
    assert np.isclose((u * Lv).sum(), (Lu * v).sum(), rtol=1e-12)
    assert (u * Lu).sum() < 0


# -------------------------------------------------------- anisotropy (Eq. 8) + constants
def test_golden_constants():
    gd = json.load(open(GOLDEN))
    e = gd["exch_prefactor_nm2"]
    exch = 2 * e["inputs"]["A_J_per_m"] / (MU0 * e["inputs"]["Ms_A_per_m"] ** 2) * 1e18
    assert abs(exch / e["value"] - 1) < e["rel_tol"]
    # The oracle's exchange prefactor (A/m per unit Laplacian of m, per 1/delta^2) equals
    # Ms * exch of the script.
    pb = oracle.Problem(3, 1, 1, 1e-9, Ms=8e5, A=1.3e-11)
    m = np.zeros(pb.shape)
    m[0, 0, 0, 1] = 1.0
    h = oracle.exchange(pb, m)[0, 0, 0, 0]          # neighbour difference of 1
    assert abs(h / (pb.Ms * e["value"] * 1e-18 / pb.cell ** 2) - 1) < e["rel_tol"]
    # reversal field of Sec. 3 in kA/m (script) vs mT (text)
    r = gd["reversal_field"]
    apm = np.array(r["script_kApm"]) * 1e3
    assert np.allclose(apm * MU0 * 1e3, r["text_mT"], atol=r["abs_tol_mT"])
    assert np.allclose(mT_to_Apm(r["text_mT"]) / 1e3, r["script_kApm"], atol=0.05)
    # gyromagnetic ratio: 0.221 /ns per kA/m == 2.21e5 m/(A s)
    gm = gd["gamma_script"]
    assert np.isclose(gm["value_per_ns_per_kApm"] * 1e9 / 1e3, gm["si_m_per_A_s"])
    # anisotropy: H_anis 100 kA/m with Ms 1000 kA/m means Ku = mu0 Ms H_K / 2.
    a = gd["sp3_anisotropy"]
    Ms = a["Ms_kApm"] * 1e3
    Ku = MU0 * Ms * a["H_anis_kApm"] * 1e3 / 2
    pb = oracle.Problem(1, 1, 1, 1e-9, Ms=Ms, Ku=Ku)
    m = np.array([0.8, 0.6, 0.0]).reshape(3, 1, 1, 1)
    h = oracle.anisotropy(pb, m).reshape(3)
    assert np.allclose(h, [a["H_anis_kApm"] * 1e3 * 0.8, 0, 0], rtol=1e-14)


# ----------------------------------------------- field = -dE/(mu0 dM) (Eq. 3) by FD
@pytest.mark.parametrize("ku", [0.0, 3.0e4])
def test_field_is_energy_derivative(ku):
    # Central differences of the Eq. 1 energy give -mu0 V Ms H.  With Ku = 0 the whole
    # field must match; the anisotropy form of Listing 2 differs from -dE/dM by a
    # field parallel to m, so with Ku != 0 the torque m x H must match.
    pb = oracle.Problem(4, 3, 2, 4e-9, Ms=8e5, A=1.3e-11, Ku=ku,
                        hext=tuple(mT_to_Apm([3.0, -7.0, 11.0])))
    m = random_unit_m(pb.shape, 5)
    V = pb.cell ** 3
    h_num = np.zeros(pb.shape)
    eps = 1e-6
    for idx in np.ndindex(*pb.shape):
        mp, mm = m.copy(), m.copy()
        mp[idx] += eps
        mm[idx] -= eps
        dE = (oracle.energy(pb, mp)[4] - oracle.energy(pb, mm)[4]) / (2 * eps)
        h_num[idx] = -dE / (MU0 * V * pb.Ms)
    h = oracle.heff_terms(pb, m)["eff"]
    scale = np.abs(h).max()
    if ku == 0.0:
        assert np.abs(h_num - h).max() / scale < 1e-7
    tq = np.cross(m, h, axis=0)
    tq_num = np.cross(m, h_num, axis=0)
    assert np.abs(tq - tq_num).max() / scale < 1e-7


def test_exchange_energy_pairs_equal_field_form():
    pb = oracle.Problem(5, 4, 3, 3e-9, Ku=0.0, demag=False)
    m = random_unit_m(pb.shape, 6)
    e = oracle.energy(pb, m)[0]
    hx = oracle.exchange(pb, m)
    e2 = -0.5 * MU0 * pb.cell ** 3 * pb.Ms * (m * hx).sum()
    assert np.isclose(e, e2, rtol=1e-12)


# ------------------------------------------------------------------- LLG (Eq. 2)
def test_rhs_orthogonal_and_vanishes_for_parallel_field():
    pb = oracle.Problem(4, 3, 2, 3e-9, alpha=0.3)
    m = random_unit_m(pb.shape, 7)
    g = np.random.default_rng(8)
    h = g.standard_normal(pb.shape) * 1e5
    f = oracle.llg_rhs(pb, m, h)
    assert np.abs((f * m).sum(axis=0)).max() < 1e-9 * np.abs(f).max()
    f0 = oracle.llg_rhs(pb, m, 3.7e4 * m)
    assert np.abs(f0).max() < 1e-14 * pb.gamma * 3.7e4


def macrospin_closed_form(theta0, phi0, H, alpha, gamma, t):
    gp = gamma / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * gp * H * t))
    ph = phi0 + gp * H * t
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_macrospin_rk4_matches_closed_form_fourth_order():
    # One cell: exchange vanishes and the demag field -M/3 is parallel to m, so m
    # precesses and relaxes about H_ext = H z exactly as the textbook LL solution.
    H = 2.0e5
    alpha = 0.1
    pb = oracle.Problem(1, 1, 1, 5e-9, Ku=0.0, alpha=alpha, hext=(0.0, 0.0, H))
    th0, ph0 = 2.5, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    T = 2e-10
    errs = []
    for nsteps in (200, 400, 800):
        m = oracle.rk4(pb, m0.reshape(3, 1, 1, 1), T / nsteps, nsteps).reshape(3)
        errs.append(np.abs(m - macrospin_closed_form(th0, ph0, H, alpha, pb.gamma, T)).max())
    assert errs[-1] < 1e-8
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_norm_preserved_and_energy_decreases():
    pb = oracle.Problem(8, 4, 2, 5e-9, Ku=500.0, alpha=0.5,
                        hext=tuple(mT_to_Apm([5.0, 0.0, -2.0])))
    m = random_unit_m(pb.shape, 9)
    e_prev = oracle.energy(pb, m)[4]
    for _ in range(20):
        m = oracle.rk4(pb, m, 1e-13, 1)
        n = np.sqrt((m * m).sum(axis=0))
        assert np.abs(n - 1).max() < 4e-16
        e = oracle.energy(pb, m)[4]
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e


def test_energy_rate_matches_dissipation():
    # dE/dt = -mu0 V Ms sum H . dm/dt = -mu0 V Ms alpha gamma/(1+alpha^2) sum |m x H|^2.
    pb = oracle.Problem(6, 4, 2, 5e-9, Ku=500.0, alpha=0.4,
                        hext=tuple(mT_to_Apm([5.0, 2.0, -2.0])))
    m = random_unit_m(pb.shape, 10)
    dt = 2e-15
    # backward/forward RK4 around t: integrate with -dt via time reversal is not LLG,
    # so use E(t+dt) - E(t) and E(t+2dt) - E(t+dt) (second-order one-sided estimate).
    m1 = oracle.rk4(pb, m, dt, 1)
    m2 = oracle.rk4(pb, m1, dt, 1)
    e0, e1, e2 = (oracle.energy(pb, x)[4] for x in (m, m1, m2))
    dEdt = (-3 * e0 + 4 * e1 - e2) / (2 * dt)
    h = oracle.heff_terms(pb, m)["eff"]
    t = np.cross(m, h, axis=0)
    V = pb.cell ** 3
    expect = -MU0 * V * pb.Ms * pb.alpha * pb.gamma / (1 + pb.alpha ** 2) * (t * t).sum()
    assert abs(dEdt / expect - 1) < 1e-3


# ------------------------------------------------------ adjoint of RK4 + renormalisation
def _loss(pb, m0, dt, n, w):
    return float((oracle.rk4(pb, m0, dt, n) * w).sum())


@pytest.mark.parametrize("periodic", [(False, False, False), (True, True, False), (True, False, True)])
def test_oracle_adjoint_matches_finite_differences(periodic):
    # The discrete adjoint (dLoss/dKu, dLoss/dm0) of n RK4 steps against central
    # differences of the forward run in FP64, for a linear loss sum(w * m_n); also
    # with periodic axes (wrapped exchange, image-summed demag).
    g = np.random.default_rng(21)
    nx, ny, nz = 5, 4, 2
    ku = 500.0 + 50.0 * g.standard_normal((nz, ny, nx))
    kw = dict(periodic=periodic, images=1)
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.3, ku_map=ku,
                        hext=tuple(mT_to_Apm([8.0, -3.0, 5.0])), **kw)
    m0 = random_unit_m(pb.shape, 22)
    w = g.standard_normal(pb.shape)
    dt, n = 1e-13, 6
    dku, dm0 = oracle.rk4_adjoint(pb, m0, dt, n, w)
    for trial in range(3):
        v = g.standard_normal(ku.shape)
        eps = 2.0
        pb_p = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.3, ku_map=ku + eps * v, hext=pb.hext, **kw)
        pb_m = oracle.Problem(nx, ny, nz, 5e-9, Ku=0.0, alpha=0.3, ku_map=ku - eps * v, hext=pb.hext, **kw)
        fd = (_loss(pb_p, m0, dt, n, w) - _loss(pb_m, m0, dt, n, w)) / (2 * eps)
        ad = float((dku * v).sum())
        assert abs(fd - ad) <= 1e-6 * abs(ad), (trial, fd, ad)
        vm = g.standard_normal(pb.shape)
        em = 1e-6
        fdm = (_loss(pb, m0 + em * vm, dt, n, w) - _loss(pb, m0 - em * vm, dt, n, w)) / (2 * em)
        adm = float((dm0 * vm).sum())
        assert abs(fdm - adm) <= 1e-6 * abs(adm), (trial, fdm, adm)


def test_macrospin_euler_first_order():
    # The appendix script's explicit Euler + renormalisation converges at first order to
    # the closed-form macrospin trajectory (halving dt halves the error).
    H, alpha = 2.0e5, 0.1
    pb = oracle.Problem(1, 1, 1, 5e-9, Ku=0.0, alpha=alpha, hext=(0.0, 0.0, H))
    th0, ph0 = 2.5, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    T = 1e-10
    errs = []
    for nsteps in (2000, 4000, 8000):
        m = oracle.euler(pb, m0.reshape(3, 1, 1, 1), T / nsteps, nsteps).reshape(3)
        errs.append(np.abs(m - macrospin_closed_form(th0, ph0, H, alpha, pb.gamma, T)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, errs


def rot(axis: int, ang: float) -> np.ndarray:
    """Right-handed rotation by ang about coordinate axis 0, 1 or 2."""
    c, s = np.cos(ang), np.sin(ang)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R = np.eye(3)
    R[i, i], R[i, j], R[j, i], R[j, j] = c, -s, s, c
    return R


def test_schedule_macrospin_piecewise_fields_closed_form():
    # Undamped single cell: each piece rotates m about its field by gamma |H| t
    # (right-handed; the demag field -M/3 is parallel to m).  Pieces along z, then x,
    # then a ramp along y: within step k of the ramp the field is H0 + (H1 - H0) k / n,
    # so after n' steps the angle is gamma dt (n' H0 + (H1 - H0) n'(n'-1) / (2 n)).
    # Rows every 7 steps across the piece boundaries.
    g = 2.211e5
    pb = oracle.Problem(1, 1, 1, 5e-9, alpha=0.0, gamma=g)
    m0 = np.array([0.6, 0.0, 0.8])
    dt, Hz, Hx, H0, H1 = 2e-14, 3.0e5, 1.5e5, 2.0e5, -1.0e5
    pieces = [(30, (0, 0, Hz), (0, 0, Hz), 0.0), (25, (Hx, 0, 0), (Hx, 0, 0), 0.0),
              (40, (0, H0, 0), (0, H1, 0), 0.0)]
    rows, mf = oracle.schedule(pb, m0.reshape(3, 1, 1, 1), pieces, dt, 7)
    assert rows.shape == (95 // 7, 4)

    def exact(t_steps):
        R = np.eye(3)
        left = t_steps
        for axis, n, ang in ((2, 30, lambda k: g * dt * Hz * k), (0, 25, lambda k: g * dt * Hx * k),
                             (1, 40, lambda k: g * dt * (k * H0 + (H1 - H0) * k * (k - 1) / (2 * 40)))):
            k = min(left, n)
            R = rot(axis, ang(k)) @ R
            left -= k
        return R @ m0

    for r in rows:
        k = int(round(r[0] / dt))
        assert np.abs(r[1:] - exact(k)).max() < 1e-9, (k, r[1:], exact(k))
    assert np.abs(mf.reshape(3) - exact(95)).max() < 1e-9
    assert pb.hext == (0.0, 0.0, 0.0) and pb.alpha == 0.0


def test_schedule_damping_switch_closed_form():
    # Single cell in H z: alpha 1 for the first piece, 0.02 for the second; the polar
    # angle follows tan(th/2) = tan(th0/2) exp(-alpha gamma' H t) per piece, the azimuth
    # gamma' H t (gamma' = gamma / (1 + alpha^2)); rows every 10 steps.
    g, H, dt = 2.211e5, 2.0e5, 1e-14
    pb = oracle.Problem(1, 1, 1, 5e-9, gamma=g)
    th0, ph0 = 2.5, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    pieces = [(200, (0, 0, H), (0, 0, H), 1.0), (300, (0, 0, H), (0, 0, H), 0.02)]
    rows, _ = oracle.schedule(pb, m0.reshape(3, 1, 1, 1), pieces, dt, 10)
    assert rows.shape == (50, 4)
    T1 = 200 * dt
    th1 = macrospin_closed_form(th0, ph0, H, 1.0, g, T1)
    th1, ph1 = np.arccos(th1[2]), np.arctan2(th1[1], th1[0])
    for r in rows:
        t = r[0]
        want = (macrospin_closed_form(th0, ph0, H, 1.0, g, t) if t <= T1 + 1e-20
                else macrospin_closed_form(th1, ph1, H, 0.02, g, t - T1))
        assert np.abs(r[1:] - want).max() < 1e-9, (t, r[1:], want)


def test_schedule_euler_rotates_by_arctan():
    # Explicit Euler + renormalisation of an undamped single cell turns m about H by
    # exactly atan(gamma |H| dt) per step (m + dt w x m has length sec of that angle for
    # the in-plane part): a closed form of the appendix update at any dt.
    g, H, dt = 2.211e5, 4.0e5, 5e-15
    pb = oracle.Problem(1, 1, 1, 3e-9, alpha=0.0, gamma=g)
    m0 = np.array([1.0, 0.0, 0.0])
    rows, _ = oracle.schedule(pb, m0.reshape(3, 1, 1, 1), [(1000, (0, 0, H), (0, 0, H), 0.0)],
                              dt, 100, method="euler")
    for r in rows:
        k = int(round(r[0] / dt))
        want = rot(2, k * np.arctan(g * H * dt)) @ m0
        assert np.abs(r[1:] - want).max() < 1e-12, (k, r[1:], want)


# ------------------------------------------------ Newell's cell-averaged tensor
def aharoni_dz(a: float, b: float, c: float) -> float:
    """Magnetometric demagnetising factor along z of a uniformly magnetised
    rectangular prism of edges 2a x 2b x 2c (Aharoni, J. Appl. Phys. 83, 3432,
    1998): an independent closed form for the cell sums of the averaged tensor."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((ab + a) / (ab - a)) + a / (2 * c) * np.log((ab + b) / (ab - b))
         + c / (2 * a) * np.log((bc - b) / (bc + b)) + c / (2 * b) * np.log((ac - a) / (ac + a))
         + 2 * np.arctan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / np.pi


def test_aharoni_closed_form_sanity():
    assert abs(aharoni_dz(1, 1, 1) - 1 / 3) < 1e-14
    for a, b, c in ((3, 1.5, 1), (1, 2, 3), (5, 1, 0.4)):
        tot = aharoni_dz(a, b, c) + aharoni_dz(b, c, a) + aharoni_dz(c, a, b)
        assert abs(tot - 1) < 1e-13


def test_newell_origin_trace_and_parity():
    k0 = oracle.newell_point(0, 0, 0)
    assert np.abs(k0 - np.array([-1 / 3, 0, 0, -1 / 3, 0, -1 / 3])).max() < 1e-15
    g = np.random.default_rng(12)
    offs = [(1, 0, 0), (1, 1, 0), (1, 1, 1), (0, 2, 1)] + [tuple(g.integers(-9, 10, 3)) for _ in range(12)]
    for d in offs:
        if d == (0, 0, 0):
            continue
        k = oracle.newell_point(*d)
        # the averaged field of one cell has zero divergence outside it: trace 0 for
        # every pair of distinct (non-overlapping) cells
        assert abs(k[0] + k[3] + k[5]) < 1e-15 * max(1.0, np.abs(k).max()), d
        assert np.array_equal(k, oracle.newell_point(-d[0], -d[1], -d[2])) or \
            np.abs(k - oracle.newell_point(-d[0], -d[1], -d[2])).max() < 1e-17
        # xy odd in y alone, xz odd in z alone
        km = oracle.newell_point(d[0], -d[1], d[2])
        assert abs(km[1] + k[1]) < 1e-17 and abs(km[0] - k[0]) < 1e-17


def test_newell_box_factors_match_aharoni():
    # Uniform m along each axis in an a x b x c box of cells: the cell average of
    # sum_j K(r_j - r_i) is minus the prism's demagnetising factor, exactly, because the
    # averaged tensor integrates the field over every cell.
    for nx, ny, nz in ((4, 4, 4), (6, 3, 2), (10, 3, 1), (5, 7, 3)):
        tab = oracle.newell_table(nx, ny, nz)
        I = np.abs(np.arange(-(nx - 1), nx))
        J = np.abs(np.arange(-(ny - 1), ny))
        K = np.abs(np.arange(-(nz - 1), nz))
        cnt = (nz - K)[:, None, None] * (ny - J)[None, :, None] * (nx - I)[None, None, :]
        N = nx * ny * nz
        dxx, dyy, dzz = (-(tab[c] * cnt).sum() / N for c in (0, 3, 5))
        a, b, c = nx / 2, ny / 2, nz / 2
        assert abs(dzz - aharoni_dz(a, b, c)) < 1e-12, (nx, ny, nz, dzz, aharoni_dz(a, b, c))
        assert abs(dxx - aharoni_dz(b, c, a)) < 1e-12
        assert abs(dyy - aharoni_dz(c, a, b)) < 1e-12
        assert abs(dxx + dyy + dzz - 1) < 1e-12


def test_newell_approaches_point_tensor_at_fourth_order():
    # Both tensors are cube averages of the dipole kernel (Newell over source and target,
    # Eqs. 10-11 over the source only); the kernel is harmonic, so the averages differ
    # from each other by O((delta / r)^4): doubling r divides the gap by ~16.
    for u in ((1, 0, 0), (2, 1, 0), (3, 2, 1)):
        gaps = []
        for s in (4, 8, 16):
            d = tuple(s * v for v in u)
            kp, kn = oracle.tensor_point(*d), oracle.newell_point(*d)
            gaps.append(np.abs(kn - kp).max() / np.abs(kp).max())
        r1, r2 = gaps[0] / gaps[1], gaps[1] / gaps[2]
        assert 13 < r1 < 19 and 14 < r2 < 18, (u, gaps)


# ------------------------------------------------------- mean of m on many cells
def test_mean_m_of_a_plane_wave_along_x_vanishes():
    # m = (cos 2 pi i/nx, sin 2 pi i/nx, 0): the roots of unity sum to zero along every
    # row, so <m> = 0 on any ny x nz (a cell counted twice or a wrong stride breaks it).
    nx, ny, nz = 6, 5, 3
    pb = oracle.Problem(nx, ny, nz, 3e-9)
    th = 2 * np.pi * np.arange(nx) / nx
    m = np.zeros(pb.shape)
    m[0] = np.cos(th)[None, None, :]
    m[1] = np.sin(th)[None, None, :]
    assert np.abs(oracle.mean_m(pb, m)).max() < 1e-15


def test_mean_m_of_cell_blocks_counts_every_cell_once():
    # 4 x 3 x 2 cells: plane k = 0 along +z (12 cells), plane k = 1 along +x for
    # i < 2 (6 cells) and along -y for i >= 2 (6 cells): <m> = (1/4, -1/4, 1/2).
    # Each component has its own value, so a planar/interleaved mix-up or a
    # divisor of one plane instead of all cells gives a different result.
    nx, ny, nz = 4, 3, 2
    pb = oracle.Problem(nx, ny, nz, 3e-9)
    m = np.zeros(pb.shape)
    m[2, 0] = 1.0
    m[0, 1, :, :2] = 1.0
    m[1, 1, :, 2:] = -1.0
    assert np.array_equal(oracle.mean_m(pb, m), np.array([0.25, -0.25, 0.5]))


# ------------------------------------------------------------ max torque |m x H|
def test_max_torque_of_cells_in_a_uniform_field():
    # No exchange, no anisotropy, no demag: the torque of cell c is |H| sin(theta_c),
    # theta_c its angle to H_ext; the largest angle below pi/2 wins.
    H = 3.0e4
    pb = oracle.Problem(5, 2, 1, 3e-9, A=0.0, Ku=0.0, demag=False, hext=(0.0, 0.0, H))
    th = np.array([0.1, 0.4, 1.2, 0.7, 2.9, 0.0, 3.1, 0.2, 1.0, 0.5]).reshape(1, 2, 5)
    m = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)])
    assert np.isclose(oracle.max_torque(pb, m), H * np.sin(1.2), rtol=1e-14)


def test_max_torque_of_a_single_cell_ignores_its_own_demag():
    # One cell: H_d = -M/3 is parallel to m (torque-free), so only H_ext acts.
    H = 5.0e4
    pb = oracle.Problem(1, 1, 1, 5e-9, Ku=0.0, hext=(H, 0.0, 0.0))
    th = 0.83
    m = np.array([np.cos(th), np.sin(th), 0.0]).reshape(3, 1, 1, 1)
    assert np.isclose(oracle.max_torque(pb, m), H * np.sin(th), rtol=1e-12)


def test_max_torque_sets_the_largest_llg_rate():
    # For a unit m the two terms of Eq. 2 are orthogonal and of equal size, so
    # |dm/dt| = gamma / sqrt(1 + alpha^2) |m x H| cell by cell, with every term of
    # the effective field present.
    pb = oracle.Problem(7, 5, 3, 4e-9, Ku=3.0e4, alpha=0.35,
                        hext=tuple(mT_to_Apm([8.0, -3.0, 5.0])))
    m = random_unit_m(pb.shape, 12)
    f = oracle.llg_rhs(pb, m, oracle.heff_terms(pb, m)["eff"])
    rate = np.sqrt((f * f).sum(axis=0)).max()
    assert np.isclose(oracle.max_torque(pb, m) * pb.gamma / np.sqrt(1 + pb.alpha ** 2), rate,
                      rtol=1e-12)


def test_sampled_euler_recipe_equals_oracle_euler():
    # The per-cell recipe the full-film GPU test applies at sampled cells (direct-sum
    # demag there, exchange, anisotropy, applied field, right-hand side on a 1-D problem
    # of the sampled cells, step, renormalisation) equals the oracle's Euler step.
    pb = oracle.Problem(12, 8, 3, 3e-9, Ms=8e5, A=1.3e-11, Ku=500.0, alpha=0.1, gamma=2.211e5,
                        hext=(1e3, -2e3, 5e2))
    m0 = random_unit_m(pb.shape, seed=1)
    obs = np.array([0, 5, 17, 100, 287])
    h = oracle.demag(pb, m0, obs) + oracle.exchange(pb, m0).reshape(3, -1)[:, obs] + \
        oracle.anisotropy(pb, m0).reshape(3, -1)[:, obs] + np.asarray(pb.hext).reshape(3, 1)
    n = len(obs)
    ps = oracle.Problem(n, 1, 1, pb.cell, Ms=pb.Ms, A=pb.A, Ku=pb.Ku, alpha=pb.alpha, gamma=pb.gamma,
                        hext=pb.hext)
    m0s = m0.reshape(3, -1)[:, obs]
    k = oracle.llg_rhs(ps, m0s.reshape(3, 1, 1, n), h.reshape(3, 1, 1, n)).reshape(3, n)
    v = m0s + 5e-14 * k
    ref = v / np.sqrt((v * v).sum(axis=0))
    full = oracle.euler(pb, m0, 5e-14, 1).reshape(3, -1)[:, obs]
    assert np.abs(ref - full).max() <= 1e-15
    assert np.abs(full - m0s).max() > 1e-3   # the step moves m
