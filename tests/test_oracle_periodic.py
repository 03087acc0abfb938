"""Pins of the oracle's periodic boundary (the alternative to zero padding named in
Sec. 2.3; the image window is the reading stated in oracle.tensor_table_periodic).

- A uniformly magnetised periodic box: the demag sum over all cells and images is
  the point field of the union prism at the observer (the eight-corner form of
  Eqs. 10-11 telescopes over adjacent cells), two half-weighted prisms along an
  axis of even period.  Written here from the prism corners, independently of
  the oracle's cell-by-cell table.
- The infinite-film limit: a film periodic in x and y, magnetised along z, has
  N_zz -> 1 and, magnetised in-plane, N_xx -> 0 as images are added.
- A spin wave along a periodic axis is an eigenvector of the exchange stencil
  with eigenvalue 2 cos(2 pi k / n) - 2.
- Cyclic shifts along periodic axes commute with the demag field, and the
  periodic table keeps the parity of every component.
- The exchange energy (Eq. 1, summed over neighbour pairs) equals
  -(mu0/2) delta^3 sum M . H_ex of the wrapped field, and the demag energy
  -(mu0/2) delta^3 sum M . H_d.
"""
import itertools

import numpy as np
import pytest

import oracle

MS = 8.0e5


def prism_tensor(lo, hi):
    """Point field tensor (6 components, order xx xy xz yy yz zz, sign of Eqs. 12-13)
    at the origin of the uniformly magnetised prism of cells lo..hi (inclusive
    integer offsets per axis, cell edge 1): corners at lo - 1/2 and hi + 1/2."""
    xs = (lo[0] - 0.5, hi[0] + 0.5)
    ys = (lo[1] - 0.5, hi[1] + 0.5)
    zs = (lo[2] - 0.5, hi[2] + 0.5)

    def lzr(a, b, c, r):   # ln(c + r), without cancellation for c < 0
        return np.log(c + r) if c >= 0 else np.log((a * a + b * b) / (r - c))

    t = np.zeros(6)
    for i, j, k in itertools.product((0, 1), repeat=3):
        X, Y, Z = xs[i], ys[j], zs[k]
        r = np.sqrt(X * X + Y * Y + Z * Z)
        s = -1.0 if (i + j + k) % 2 else 1.0
        t[0] += s * np.arctan(Y * Z / (X * r))
        t[3] += s * np.arctan(X * Z / (Y * r))
        t[5] += s * np.arctan(X * Y / (Z * r))
        t[1] -= s * lzr(X, Y, Z, r)
        t[2] -= s * lzr(X, Z, Y, r)
        t[4] -= s * lzr(Y, Z, X, r)
    return t / (4 * np.pi)


def axis_windows(n, periodic, images, o):
    """[(lo, hi, weight)] of source offsets seen from observer coordinate o."""
    if not periodic:
        return [(-o, n - 1 - o, 1.0)]
    if n % 2:
        h = (n - 1) // 2
        return [(-h - images * n, h + images * n, 1.0)]
    h = n // 2
    return [(-h - images * n, h - 1 + images * n, 0.5), (-h + 1 - images * n, h + images * n, 0.5)]


def apply(t, m):
    xx, xy, xz, yy, yz, zz = t
    return np.array([xx * m[0] + xy * m[1] + xz * m[2], xy * m[0] + yy * m[1] + yz * m[2],
                     xz * m[0] + yz * m[1] + zz * m[2]])


@pytest.mark.parametrize("dims,periodic,images", [
    ((6, 5, 3), (True, True, False), 0),
    ((6, 5, 3), (True, True, False), 2),
    ((5, 4, 2), (True, False, True), 1),
    ((4, 4, 4), (True, True, True), 1),
    ((7, 1, 3), (False, True, True), 3),
])
def test_uniform_periodic_box_is_the_union_prism(dims, periodic, images):
    nx, ny, nz = dims
    pb = oracle.Problem(nx, ny, nz, 5e-9, Ms=MS, periodic=periodic, images=images)
    u = np.array([0.3, -0.5, 0.81])
    u /= np.linalg.norm(u)
    m = np.broadcast_to(u.reshape(3, 1, 1, 1), pb.shape).copy()
    h = oracle.demag(pb, m)
    worst = 0.0
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        ref = np.zeros(3)
        for (lx, hx, wx) in axis_windows(nx, periodic[0], images, i):
            for (ly, hy, wy) in axis_windows(ny, periodic[1], images, j):
                for (lz, hz, wz) in axis_windows(nz, periodic[2], images, k):
                    ref += wx * wy * wz * MS * apply(prism_tensor((lx, ly, lz), (hx, hy, hz)), u)
        worst = max(worst, np.abs(h[:, k, j, i] - ref).max() / MS)
    assert worst < 1e-12, worst


def test_periodic_film_tends_to_the_infinite_slab():
    # N_zz -> 1 (H_z -> -M_z) and N_xx -> 0 as the lateral images grow
    dev_z, dev_x = [], []
    for images in (0, 1, 2, 4, 8):
        pb = oracle.Problem(8, 8, 2, 5e-9, Ms=MS, periodic=(True, True, False), images=images)
        mz = np.zeros(pb.shape)
        mz[2] = 1.0
        mx = np.zeros(pb.shape)
        mx[0] = 1.0
        dev_z.append(abs(1.0 + oracle.demag(pb, mz)[2].mean() / MS))
        dev_x.append(abs(oracle.demag(pb, mx)[0].mean() / MS))
    assert all(b < a for a, b in zip(dev_z, dev_z[1:])), dev_z
    assert all(b < a for a, b in zip(dev_x, dev_x[1:])), dev_x
    # a slab 2 cells thick and 17 x 8 = 136 cells wide: edge effects of order 2/136
    assert dev_z[-1] < 0.02 and dev_x[-1] < 0.02


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_periodic_spin_wave_is_an_exchange_eigenvector(axis):
    n = (12, 9, 10)
    periodic = [False, False, False]
    periodic[axis] = True
    pb = oracle.Problem(*n, 4e-9, Ms=MS, A=1.3e-11, periodic=tuple(periodic))
    k = 2
    pos = np.indices((n[2], n[1], n[0]))[2 - axis]        # coordinate along `axis`
    th = 2 * np.pi * k * pos / n[axis]
    m = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)])
    h = oracle.exchange(pb, m)
    pref = 2 * pb.A / (oracle.MU0 * MS * pb.cell ** 2)
    lam = 2 * np.cos(2 * np.pi * k / n[axis]) - 2
    assert np.abs(h - pref * lam * m).max() <= 1e-9 * pref


def test_cyclic_shift_commutes_with_periodic_demag():
    pb = oracle.Problem(6, 5, 4, 5e-9, Ms=MS, periodic=(True, True, False), images=1)
    g = np.random.default_rng(3)
    m = g.standard_normal(pb.shape)
    m /= np.linalg.norm(m, axis=0)
    h = oracle.demag(pb, m)
    for sx, sy in ((1, 0), (0, 2), (3, 4)):
        hs = oracle.demag(pb, np.roll(m, (sy, sx), axis=(2, 3)))
        assert np.abs(hs - np.roll(h, (sy, sx), axis=(2, 3))).max() < 1e-9 * MS


@pytest.mark.parametrize("n", [6, 7])
def test_periodic_table_keeps_component_parities(n):
    # xy odd in x and y, xz odd in x and z, yz odd in y and z, diagonal even
    t = oracle.tensor_table_periodic(n, n, n, (True, True, True), images=1)
    par = {0: (1, 1, 1), 1: (-1, -1, 1), 2: (-1, 1, -1), 3: (1, 1, 1), 4: (1, -1, -1), 5: (1, 1, 1)}
    rev = (-np.arange(n)) % n
    for c, (sx, sy, sz) in par.items():
        tc = t[c]
        assert np.allclose(tc[:, :, rev], sx * tc, atol=1e-15)
        assert np.allclose(tc[:, rev, :], sy * tc, atol=1e-15)
        assert np.allclose(tc[rev, :, :], sz * tc, atol=1e-15)


@pytest.mark.parametrize("periodic", [(True, False, False), (True, True, False), (False, True, True),
                                      (True, True, True)])
def test_periodic_energy_matches_its_fields(periodic):
    pb = oracle.Problem(5, 2, 3, 4e-9, Ms=MS, A=1.3e-11, Ku=2e3, periodic=periodic, images=1)
    g = np.random.default_rng(8)
    m = g.standard_normal(pb.shape)
    m /= np.linalg.norm(m, axis=0)
    e = oracle.energy(pb, m)
    V = pb.cell ** 3
    e_ex = -0.5 * oracle.MU0 * V * MS * (m * oracle.exchange(pb, m)).sum()
    e_d = -0.5 * oracle.MU0 * V * MS * (m * oracle.demag(pb, m)).sum()
    assert abs(e[0] - e_ex) <= 1e-12 * abs(e_ex)
    assert abs(e[2] - e_d) <= 1e-12 * abs(e_d)
