"""FP64 CPU oracle for the micromagnetic LLG step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package; the product path (``paper_1501_07293_amd``) never does, and the
two share no code.  The arithmetic lives in ``mmag_oracle.c`` (plain C, FP64,
OpenMP over observation cells); this module builds it with gcc and marshals
numpy arrays.  Paper: Zhu, arXiv:1501.07293 -- Sec. 2 Eqs. 1-3 (energy, LLG,
effective field), Sec. 2.1 Eqs. 5-7 (exchange, Neumann boundary), Sec. 2.2
Eq. 8 (anisotropy), Sec. 2.3 Eqs. 10-13 (demag tensor and direct sum).

Layout: m and fields are float64 arrays of shape (3, nz, ny, nx), x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mmag_oracle.c")
_SRC_NEWELL = os.path.join(_HERE, "newell_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MU0 = 4.0e-7 * np.pi


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, IEEE FP64 (binary128 for Newell's tensor),
    no fast-math, OpenMP)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_NEWELL))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu99",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, _SRC_NEWELL, "-o", tmp,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("cell", ctypes.c_double), ("Ms", ctypes.c_double), ("A", ctypes.c_double),
                ("Ku", ctypes.c_double), ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("hext", ctypes.c_double * 3), ("ku_map", ctypes.POINTER(ctypes.c_double)),
                ("demag", ctypes.c_int32), ("periodic", ctypes.c_int32 * 3), ("images", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.or_tensor_point.argtypes = [ctypes.c_int32] * 3 + [dp]
        lib.or_tensor_table.argtypes = [ctypes.c_int32] * 3 + [dp]
        lib.or_newell_point.argtypes = [ctypes.c_int32] * 3 + [dp]
        lib.or_newell_table.argtypes = [ctypes.c_int32] * 3 + [dp]
        lib.or_tensor_table_periodic.argtypes = ([ctypes.c_int32] * 3 + [ctypes.POINTER(ctypes.c_int32)]
                                                 + [ctypes.c_int32] * 2 + [dp])
        lib.or_demag.argtypes = [pp, dp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        lib.or_exchange.argtypes = [pp, dp, dp]
        lib.or_anisotropy.argtypes = [pp, dp, dp]
        lib.or_heff.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        lib.or_llg_rhs.argtypes = [pp, dp, dp, dp]
        lib.or_rk4.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int64]
        lib.or_energy.argtypes = [pp, dp, dp, dp]
        lib.or_mean_m.argtypes = [pp, dp, dp]
        lib.or_max_torque.argtypes = [pp, dp, dp]
        lib.or_max_torque.restype = ctypes.c_double
        lib.or_rk4_adjoint.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int64, dp, dp, dp]
        lib.or_euler.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int64]
        for f in ("or_tensor_point", "or_tensor_table", "or_tensor_table_periodic", "or_demag",
                  "or_exchange",
                  "or_anisotropy", "or_heff", "or_llg_rhs", "or_rk4", "or_energy", "or_mean_m",
                  "or_rk4_adjoint", "or_euler"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """Grid + material in SI units (Sec. 2; the constants of Eq. 2 and Eq. 8)."""
    nx: int
    ny: int
    nz: int
    cell: float                     # m
    Ms: float = 8.0e5               # A/m
    A: float = 1.3e-11              # J/m
    Ku: float = 0.0                 # J/m^3, easy axis x
    alpha: float = 0.5
    gamma: float = 2.211e5          # m/(A s), multiplies H in A/m
    hext: Sequence[float] = (0.0, 0.0, 0.0)   # A/m
    ku_map: Optional[np.ndarray] = None       # (nz, ny, nx) J/m^3, overrides Ku
    demag: bool = True
    tensor: str = "point"           # "point": Eqs. 10-11; "newell": cell-averaged (Newell et al.)
    periodic: Sequence[bool] = (False, False, False)   # per axis x, y, z
    images: int = 0                 # periodic axes: images on each side beyond the minimum image
    _table: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (3, self.nz, self.ny, self.nx)

    def _params(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.cell, p.Ms, p.A, p.Ku = self.cell, self.Ms, self.A, self.Ku
        p.alpha, p.gamma = self.alpha, self.gamma
        for a in range(3):
            p.hext[a] = float(self.hext[a])
        if self.ku_map is not None:
            self._ku = np.ascontiguousarray(self.ku_map, dtype=np.float64).reshape(-1)
            assert self._ku.size == self.N
            p.ku_map = _dptr(self._ku)
        p.demag = 1 if self.demag else 0
        for a in range(3):
            p.periodic[a] = 1 if self.periodic[a] else 0
        p.images = int(self.images)
        return p

    def table(self) -> np.ndarray:
        """Demag tensor over all offsets: (6, 2nz-1, 2ny-1, 2nx-1); order xx,xy,xz,yy,yz,zz.
        Along a periodic axis the table has n entries, offsets mod n summed over
        images (tensor_table_periodic)."""
        if self._table is None:
            if any(self.periodic):
                self._table = tensor_table_periodic(self.nx, self.ny, self.nz, self.periodic,
                                                    self.images, self.tensor)
            else:
                make = newell_table if self.tensor == "newell" else tensor_table
                self._table = make(self.nx, self.ny, self.nz)
        return self._table


def tensor_point(I: int, J: int, K: int) -> np.ndarray:
    """Eqs. 10-11 at the integer offset (I,J,K) = source - observer; dimensionless."""
    out = np.zeros(6)
    _load().or_tensor_point(int(I), int(J), int(K), _dptr(out))
    return out


def tensor_table(nx: int, ny: int, nz: int) -> np.ndarray:
    out = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    _load().or_tensor_table(nx, ny, nz, _dptr(out))
    return out


def tensor_table_periodic(nx: int, ny: int, nz: int, periodic, images: int = 0,
                          tensor: str = "point") -> np.ndarray:
    """Tensor table with periodic axes (the boundary Sec. 2.3 contrasts with zero
    padding).  Along a periodic axis of period n the entry t (0 <= t < n) holds
    the sum of the tensor over the offsets t + j n: the representative of t
    nearest zero (both t and t - n with weight 1/2 when 2t = n) and `images`
    further multiples of n on each side; open axes as in tensor_table."""
    per = (ctypes.c_int32 * 3)(*[1 if p else 0 for p in periodic])
    dims = [n if p else 2 * n - 1 for n, p in zip((nx, ny, nz), periodic)]
    out = np.zeros((6, dims[2], dims[1], dims[0]))
    _load().or_tensor_table_periodic(nx, ny, nz, per, int(images), 1 if tensor == "newell" else 0,
                                     _dptr(out))
    return out


def newell_point(I: int, J: int, K: int) -> np.ndarray:
    """Newell's cell-averaged tensor at the integer offset (I,J,K), in the sign
    convention of Eqs. 12-13 (K = -N; K(0) = -I/3 for a cube); evaluated in
    binary128 and returned in FP64."""
    out = np.zeros(6)
    _load().or_newell_point(int(I), int(J), int(K), _dptr(out))
    return out


def newell_table(nx: int, ny: int, nz: int) -> np.ndarray:
    out = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    _load().or_newell_table(nx, ny, nz, _dptr(out))
    return out


def _m(pb: Problem, m) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.float64).reshape(pb.shape))
    return a


def demag(pb: Problem, m, obs: Optional[np.ndarray] = None) -> np.ndarray:
    """Direct-sum demag field (Eqs. 12-13), A/m.  obs: optional linear cell
    indices; then the result is (3, len(obs)), else (3, nz, ny, nx)."""
    m = _m(pb, m)
    tab = pb.table()
    p = pb._params()
    if obs is None:
        out = np.zeros(pb.shape)
        _load().or_demag(ctypes.byref(p), _dptr(m), _dptr(tab), None, 0, _dptr(out))
    else:
        o = np.ascontiguousarray(obs, dtype=np.int64)
        out = np.zeros((3, o.size))
        _load().or_demag(ctypes.byref(p), _dptr(m), _dptr(tab),
                         o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), o.size, _dptr(out))
    return out


def exchange(pb: Problem, m) -> np.ndarray:
    m = _m(pb, m)
    out = np.zeros(pb.shape)
    p = pb._params()
    _load().or_exchange(ctypes.byref(p), _dptr(m), _dptr(out))
    return out


def anisotropy(pb: Problem, m) -> np.ndarray:
    m = _m(pb, m)
    out = np.zeros(pb.shape)
    p = pb._params()
    _load().or_anisotropy(ctypes.byref(p), _dptr(m), _dptr(out))
    return out


def heff_terms(pb: Problem, m):
    """Returns dict with 'exch', 'anis', 'demag', 'ext', 'eff' fields, A/m."""
    m = _m(pb, m)
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    ex, an, dm, ef = (np.zeros(pb.shape) for _ in range(4))
    _load().or_heff(ctypes.byref(p), _dptr(m), _dptr(tab), _dptr(ex), _dptr(an), _dptr(dm),
                    _dptr(ef))
    ext = np.broadcast_to(np.asarray(pb.hext, dtype=np.float64).reshape(3, 1, 1, 1),
                          pb.shape).copy()
    return {"exch": ex, "anis": an, "demag": dm, "ext": ext, "eff": ef}


def llg_rhs(pb: Problem, m, heff) -> np.ndarray:
    m = _m(pb, m)
    h = _m(pb, heff)
    out = np.zeros(pb.shape)
    p = pb._params()
    _load().or_llg_rhs(ctypes.byref(p), _dptr(m), _dptr(h), _dptr(out))
    return out


def rk4(pb: Problem, m, dt: float, nsteps: int) -> np.ndarray:
    """Classical RK4 with per-step renormalisation; returns the new m."""
    m = _m(pb, m).copy()
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    _load().or_rk4(ctypes.byref(p), _dptr(m), _dptr(tab), float(dt), int(nsteps))
    return m


def euler(pb: Problem, m, dt: float, nsteps: int) -> np.ndarray:
    """Explicit Euler with per-step renormalisation (the appendix script's update)."""
    m = _m(pb, m).copy()
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    _load().or_euler(ctypes.byref(p), _dptr(m), _dptr(tab), float(dt), int(nsteps))
    return m


def schedule(pb: Problem, m0, pieces, dt: float, every: int, method: str = "rk4"):
    """A time-dependent protocol (Sec. 3, the switching experiment of standard
    problem #4, and the appendix script that drives it): the pieces
    (steps, h0, h1, alpha) run in order; during step n of a piece the applied
    field is h0 + (h1 - h0) n / steps (A/m) and the damping is alpha.  After
    every `every`-th step (counted over all pieces) a row (t, <m_x>, <m_y>,
    <m_z>) is recorded, t = steps done * dt.  Returns (rows (k, 4), final m).
    pb.hext and pb.alpha are restored afterwards."""
    step = rk4 if method == "rk4" else euler
    m = _m(pb, m0).copy()
    rows, done = [], 0
    keep = (tuple(pb.hext), pb.alpha)
    try:
        for steps, h0, h1, alpha in pieces:
            pb.alpha = float(alpha)
            ramp = any(float(h0[c]) != float(h1[c]) for c in range(3))
            n = 0
            while n < steps:
                run = 1 if ramp else min(steps - n, every - done % every)
                f = n / steps
                pb.hext = tuple(float(h0[c]) + (float(h1[c]) - float(h0[c])) * f for c in range(3))
                m = step(pb, m, dt, run)
                n += run
                done += run
                if done % every == 0:
                    rows.append((done * dt, *mean_m(pb, m)))
    finally:
        pb.hext, pb.alpha = keep
    return np.array(rows, dtype=np.float64).reshape(-1, 4), m


def energy(pb: Problem, m) -> np.ndarray:
    """[E_exch, E_anis, E_demag, E_zeeman, E_total] in J (Eq. 1 times the cell volume)."""
    m = _m(pb, m)
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    out = np.zeros(5)
    _load().or_energy(ctypes.byref(p), _dptr(m), _dptr(tab), _dptr(out))
    return out


def mean_m(pb: Problem, m) -> np.ndarray:
    m = _m(pb, m)
    p = pb._params()
    out = np.zeros(3)
    _load().or_mean_m(ctypes.byref(p), _dptr(m), _dptr(out))
    return out


def max_torque(pb: Problem, m) -> float:
    """max over cells of |m x H_eff| in A/m (H_eff of Eq. 3 at m)."""
    m = _m(pb, m)
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    return float(_load().or_max_torque(ctypes.byref(p), _dptr(m), _dptr(tab)))


def rk4_adjoint(pb: Problem, m0, dt: float, nsteps: int, lam_final):
    """Discrete adjoint of rk4(): given dLoss/dm at the final state, returns
    (dLoss/dKu per cell (nz, ny, nx), dLoss/dm0 (3, nz, ny, nx)).  FP64; keeps
    every stage state in memory, so for small grids."""
    m0 = _m(pb, m0)
    lam = _m(pb, lam_final)
    tab = pb.table() if pb.demag else np.zeros(1)
    p = pb._params()
    dku = np.zeros((pb.nz, pb.ny, pb.nx))
    dm0 = np.zeros(pb.shape)
    _load().or_rk4_adjoint(ctypes.byref(p), _dptr(m0), _dptr(tab), float(dt), int(nsteps),
                           _dptr(lam), _dptr(dku), _dptr(dm0))
    return dku, dm0
