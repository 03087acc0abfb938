"""Seeded synthetic inputs and the five workload configurations.

This module holds no arithmetic of the method: it only draws seeded random
numbers (numpy PCG64) and states the workload parameters.  Both the HIP path
(through its tests and the benchmark) and the oracle take their inputs from
here, so they always see identical m, fields and maps.

Workloads (stand-ins for the paper's muMAG standard problems, Sec. 3, whose
reference curves are not available): a small strip, a mid-size film driven by
a step field, a large film, a batch of uneven grids, a differentiation case
with a per-cell anisotropy map, and the standard-problem-#4 protocol of the
appendix script.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

MU0 = 4.0e-7 * np.pi


def mT_to_Apm(b_mT) -> np.ndarray:
    """Applied field given as mu0*H in mT -> H in A/m."""
    return np.asarray(b_mT, dtype=np.float64) * 1e-3 / MU0


@dataclass
class Config:
    name: str
    nx: int
    ny: int
    nz: int
    cell: float
    Ms: float = 8.0e5
    A: float = 1.3e-11
    Ku: float = 500.0
    alpha: float = 0.5
    gamma: float = 2.211e5
    hext: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # A/m
    dt: float = 1e-13
    steps: int = 1000
    pad: Tuple[int, int, int] = (0, 0, 0)               # 0 = 2n (or smallest smooth)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (3, self.nz, self.ny, self.nx)


# Small strip: 32x8x1, delta 5 nm, Ku 500 J/m^3 along x, alpha 0.5, RK4 dt 1e-13 s, 2000 steps.
SMALL = Config("small 32x8x1", 32, 8, 1, 5e-9, Ku=500.0, alpha=0.5, dt=1e-13, steps=2000)

# Mid film: 256x64x4, delta 4 nm, alpha 0.02, step field (-20, 3, 0) mT, dt 5e-14 s, 10000 steps.
MID = Config("mid film 256x64x4", 256, 64, 4, 4e-9, Ku=500.0, alpha=0.02,
             hext=tuple(mT_to_Apm([-20.0, 3.0, 0.0])), dt=5e-14, steps=10000)

# Large film: 512x512x16 (4.19M cells), delta 3 nm, Ku 0, alpha 0.1, H 0, dt 5e-14 s, 500 steps.
LARGE = Config("large film 512x512x16", 512, 512, 16, 3e-9, Ku=0.0, alpha=0.1,
               dt=5e-14, steps=500)

# Differentiation: 128x128x1, delta 5 nm, alpha 0.1, per-cell Ku map, 500 steps, dt 1e-13 s.
DIFF = Config("differentiation 128x128x1", 128, 128, 1, 5e-9, Ku=500.0, alpha=0.1,
              dt=1e-13, steps=500)

# Batched: material of the small strip, delta 5 nm, dt 1e-13 s, 1000 steps.
BATCH_TEMPLATE = Config("batched sample", 0, 0, 0, 5e-9, Ku=500.0, alpha=0.5, dt=1e-13,
                        steps=1000)


# Standard problem #4 (Sec. 3, field 1) as the appendix script sets it up: 166x42x1 cells of
# 3 nm (500 x 125 x 3 nm), Ms 800 kA/m, A 1.3e-11 J/m, no anisotropy, explicit Euler with
# dt = 5 fs for 150000 steps, m starting along +x, <m> recorded every 1000 steps.
SP4 = Config("standard problem 4 film 166x42x1", 166, 42, 1, 3e-9, Ku=0.0, alpha=0.5,
             dt=5e-15, steps=150000)


def sp4_pieces(shrink: int = 1) -> List[tuple]:
    """The appendix protocol as schedule pieces (steps, h0, h1, alpha), fields in A/m:
    steps 1..3999 a saturating 100 kA/m along each axis; 4000..5999 that field ramped
    linearly to zero (the script's step t carries (6000 - t)/20 kA/m on each axis); 6000..50000
    relaxation without field (alpha 0.5 throughout); 50001..150000 the reversing field
    (-19.576, 3.422, 0) kA/m = (-24.6, 4.3, 0) mT with alpha 0.02.  `shrink` divides every
    piece's length (quick variants of the same shape)."""
    sat = (1.0e5, 1.0e5, 1.0e5)
    zero = (0.0, 0.0, 0.0)
    rev = (-19.576e3, 3.422e3, 0.0)
    return [(3999 // shrink, sat, sat, 0.5), (2000 // shrink, sat, zero, 0.5),
            (44001 // shrink, zero, zero, 0.5), (100000 // shrink, rev, rev, 0.02)]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_unit_m(shape, seed: int) -> np.ndarray:
    """Uniform random unit vectors (normalised standard normals), float64 (3, ...)."""
    g = rng(seed)
    v = g.standard_normal(size=tuple(shape))
    return v / np.sqrt((v * v).sum(axis=0, keepdims=True))


def smooth_unit_m(shape, seed: int, modes: int = 6) -> np.ndarray:
    """Smooth, domain-like unit field: a few random low-wavenumber cosine modes
    per component, normalised.  Stand-in for a relaxed film state."""
    g = rng(seed)
    _, nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for a in range(3):
        acc = np.full((nz, ny, nx), g.normal() * (2.0 if a == 0 else 0.5))
        for _ in range(modes):
            kx, ky, kz = g.uniform(0, 3.0), g.uniform(0, 3.0), g.uniform(0, 1.0)
            ph = g.uniform(0, 2 * np.pi)
            amp = g.normal()
            acc = acc + amp * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / max(nz, 1))
                                     + ph)
        out[a] = acc
    return out / np.sqrt((out * out).sum(axis=0, keepdims=True))


def ku_map(cfg: Config, seed: int, mean: float = 500.0, sd: float = 50.0) -> np.ndarray:
    """Per-cell anisotropy map Ku = mean + N(0, sd^2), shape (nz, ny, nx), J/m^3."""
    g = rng(seed)
    return mean + sd * g.standard_normal(size=(cfg.nz, cfg.ny, cfg.nx))


def vortex_target(cfg: Config, seed: int, core: float = 10e-9) -> np.ndarray:
    """Seeded vortex-like unit field: centre jittered by +-10% of the side,
    circulation and polarity +-1, m_z = p exp(-(rho/core)^2), in-plane azimuthal."""
    g = rng(seed)
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    cx = (0.5 + g.uniform(-0.1, 0.1)) * nx * cfg.cell
    cy = (0.5 + g.uniform(-0.1, 0.1)) * ny * cfg.cell
    circ = 1.0 if g.uniform() < 0.5 else -1.0
    pol = 1.0 if g.uniform() < 0.5 else -1.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = (x + 0.5) * cfg.cell - cx
    Y = (y + 0.5) * cfg.cell - cy
    rho = np.sqrt(X * X + Y * Y) + 1e-30
    mz = pol * np.exp(-(rho / core) ** 2)
    ip = np.sqrt(np.maximum(1.0 - mz * mz, 0.0))
    m = np.stack([-circ * Y / rho * ip, circ * X / rho * ip, mz])
    return m / np.sqrt((m * m).sum(axis=0, keepdims=True))


@dataclass
class BatchSample:
    nx: int
    ny: int
    nz: int
    hext: np.ndarray      # A/m
    seed: int


def batch_samples(n: int = 512, seed: int = 0, lo: int = 32, hi: int = 128,
                  radius_mT: float = 50.0) -> List[BatchSample]:
    """Uneven grids: nx, ny uniform integers in [lo, hi], nz uniform in {1, 2};
    each sample's applied field uniform in a ball of radius_mT (as mu0 H)."""
    ss = np.random.SeedSequence(seed)
    out = []
    for q, child in enumerate(ss.spawn(n)):
        g = np.random.default_rng(child)
        nx = int(g.integers(lo, hi + 1))
        ny = int(g.integers(lo, hi + 1))
        nz = int(g.integers(1, 3))
        d = g.standard_normal(3)
        d = d / np.sqrt((d * d).sum())
        r = radius_mT * g.uniform() ** (1.0 / 3.0)
        out.append(BatchSample(nx, ny, nz, mT_to_Apm(d * r), int(g.integers(0, 2**31 - 1))))
    return out


def observation_cells(nx: int, ny: int, nz: int, n: int = 1024, seed: int = 0) -> np.ndarray:
    """Seeded sorted linear indices of at least n observation cells for sampled field
    checks: all 8 corners, 4 cells on each of the 12 edges, 16 on each of the 6 faces,
    the rest uniform over the grid (x fastest: index (k ny + j) nx + i)."""
    g = rng(seed)
    pts = []
    for k in (0, nz - 1):
        for j in (0, ny - 1):
            for i in (0, nx - 1):
                pts.append((i, j, k))
    ends = {0: (0, nx - 1), 1: (0, ny - 1), 2: (0, nz - 1)}
    size = (nx, ny, nz)
    for axis in range(3):                       # edges along `axis`
        o1, o2 = [a for a in range(3) if a != axis]
        for e1 in ends[o1]:
            for e2 in ends[o2]:
                for t in g.integers(0, size[axis], 4):
                    p = [0, 0, 0]
                    p[axis], p[o1], p[o2] = int(t), e1, e2
                    pts.append(tuple(p))
    for axis in range(3):                       # faces normal to `axis`
        o1, o2 = [a for a in range(3) if a != axis]
        for e in ends[axis]:
            for _ in range(16):
                p = [0, 0, 0]
                p[axis], p[o1], p[o2] = e, int(g.integers(0, size[o1])), int(g.integers(0, size[o2]))
                pts.append(tuple(p))
    idx = {(k * ny + j) * nx + i for i, j, k in pts}
    N = nx * ny * nz
    while len(idx) < min(n, N):
        idx.update(int(v) for v in g.integers(0, N, n - len(idx)))
    return np.array(sorted(idx), dtype=np.int64)
