"""The batched layout the benchmark runs and single grids on power-of-two padding,
against the FP64 oracle.

With power-of-two padding most grids of the 512-grid workload fill less than
half of each padded line (33 cells padded to 128, 97 to 256), so the pruned
size-specialised line transforms run with a partly filled valid half.  These
tests compare that path with the oracle's direct sum (every field term at every
cell, relative max <= 1e-5 in FP32, 1e-11 in FP64) and with its RK4 trajectory
(<= 1e-4 in m in FP32, 1e-9 in FP64), on the sizes of the batched workload and
on grids of its actual seeded draw.  The oracle gets the GPU's own normalised m.
"""
import numpy as np
import pytest

import oracle
from synthetic import BATCH_TEMPLATE, batch_samples, mT_to_Apm, random_unit_m
from tests.gpu_util import rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

C = BATCH_TEMPLATE
# sizes of the batched workload's range whose padded lines are mostly empty (2n < P)
C4_SIZES = [(33, 47, 1), (37, 128, 2), (97, 61, 1), (45, 32, 2), (128, 128, 1), (81, 70, 2)]
PADS = {"pow2": dict(pow2_pad=True), "fast": dict(fast_pad=True)}
FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}
TRAJ_TOL = {"f64": 1e-9, "f32": 1e-4}
TERMS = ("exch", "anis", "demag", "ext", "eff")


def pow2_at_least(v):
    q = 2
    while q < v:
        q <<= 1
    return q


def fast_at_least(v):
    """Powers of two and the mixed-radix lengths 96, 160, 192, 224."""
    return min([q for q in (96, 160, 192, 224) if q >= v] + [pow2_at_least(v)])


def oracle_problem(dims, hext):
    nx, ny, nz = dims
    return oracle.Problem(nx, ny, nz, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                          hext=tuple(hext))


def fields_for(n, seed):
    g = np.random.default_rng(seed)
    return mT_to_Apm(g.uniform(-40, 40, size=(n, 3)))


def check_terms(got, pb, m, precision, label):
    ref = oracle.heff_terms(pb, m)
    for term in TERMS:
        if np.abs(ref[term]).max() == 0:
            assert np.abs(got[term]).max() == 0, (label, term)
            continue
        err = rel_max(got[term], ref[term])
        assert err <= FIELD_TOL[precision], (label, term, err)


@pytest.mark.parametrize("pad", ["pow2", "fast"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims", C4_SIZES)
def test_single_grid_specialised_padding_matches_oracle(dims, precision, pad):
    # One grid with power-of-two padding, or the padding of the specialised set
    # (powers of two and the mixed-radix 96, 160, 192, 224), and the size-specialised
    # passes (the single-grid form of the batch's size classes): every field term at
    # every cell, then 20 RK4 steps.
    nx, ny, nz = dims
    hext = mT_to_Apm([14.0, -6.0, 9.0])
    pb = oracle_problem(dims, hext)
    sim = mmag.Sim(nx, ny, nz, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                   precision=precision, **PADS[pad])
    p = sim.plan()
    want = pow2_at_least if pad == "pow2" else fast_at_least
    assert (p["px"], p["py"]) == (want(2 * nx - 1), want(2 * ny - 1))
    assert p["generic_fft"] == 0
    sim.set_hext(hext)
    sim.set_m(random_unit_m(pb.shape, seed=nx * ny + nz))
    m = to_np(sim.get_m())
    check_terms({t: to_np(sim.field(t)) for t in TERMS}, pb, m, precision, dims)
    sim.step(20, C.dt)
    err = np.abs(to_np(sim.get_m()) - oracle.rk4(pb, m, C.dt, 20)).max()
    print(f"{dims} {precision} padded {p['px']}x{p['py']}x{p['pz']}: m after 20 steps {err:.2e}")
    assert err <= TRAJ_TOL[precision]


@pytest.mark.parametrize("pad", ["pow2", "fast"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_size_class_batch_matches_oracle(precision, pad):
    # The batch on power-of-two (or specialised-set) padding with the size-class
    # passes: every field term of every grid at every cell; the trajectory of every
    # grid after 20 steps, and of the grids below 10^4 cells after 200 steps.
    hext = fields_for(len(C4_SIZES), seed=51)
    m0 = [random_unit_m((3, g[2], g[1], g[0]), seed=700 + i) for i, g in enumerate(C4_SIZES)]
    b = mmag.BatchSim(C4_SIZES, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision=precision, graph=True, **PADS[pad])
    info = b.info()
    assert info[pad + "_pad"] == 1 and info["size_classes"] == 1
    b.set_m(m0)
    m_used = [to_np(x) for x in b.get_m()]
    fields = {t: [to_np(x) for x in b.field(t)] for t in TERMS}
    pbs = [oracle_problem(g, hext[i]) for i, g in enumerate(C4_SIZES)]
    for i, g in enumerate(C4_SIZES):
        check_terms({t: fields[t][i] for t in TERMS}, pbs[i], m_used[i], precision, g)
    b.step(20, C.dt)
    got = [to_np(x) for x in b.get_m()]
    ref = [oracle.rk4(pbs[i], m_used[i], C.dt, 20) for i in range(len(C4_SIZES))]
    for i, g in enumerate(C4_SIZES):
        err = np.abs(got[i] - ref[i]).max()
        print(f"{g} {precision}: m after 20 steps {err:.2e}")
        assert err <= TRAJ_TOL[precision], (g, err)
    b.step(180, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for i, g in enumerate(C4_SIZES):
        if g[0] * g[1] * g[2] >= 10000:
            continue
        err = np.abs(got[i] - oracle.rk4(pbs[i], ref[i], C.dt, 180)).max()
        print(f"{g} {precision}: m after 200 steps {err:.2e}")
        assert err <= TRAJ_TOL[precision], (g, err)


def _isprime(n):
    return n > 2 and all(n % p for p in range(2, int(n ** 0.5) + 1))


def test_autotuned_512_grid_workload_samples_match_oracle():
    # The batched workload as the benchmark builds it (512 seeded grids, autotuned
    # layout, FP32, graph replay): 8 of its grids -- the smallest, the largest and six
    # whose nx and ny are both odd primes -- against the oracle, every field term at
    # every cell and the trajectory after 10 steps.
    samples = batch_samples(512, seed=0)
    grids = [(s.nx, s.ny, s.nz) for s in samples]
    hext = np.array([s.hext for s in samples])
    m0 = [random_unit_m((3, s.nz, s.ny, s.nx), seed=s.seed) for s in samples]
    b = mmag.BatchSim(grids, C.cell, Ms=C.Ms, A=C.A, Ku=C.Ku, alpha=C.alpha, gamma=C.gamma,
                      hext=hext, precision="f32", graph=True, autotune=True)
    print("layout:", b.info())
    sizes = [g[0] * g[1] * g[2] for g in grids]
    primes = [i for i, g in enumerate(grids) if _isprime(g[0]) and _isprime(g[1])][:6]
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes))] + primes
    assert len(set(pick)) == 8
    b.set_m(m0)
    m_used = [to_np(x) for x in b.get_m()]
    fields = {t: [to_np(x) for x in b.field(t)] for t in TERMS}
    b.step(10, C.dt)
    got = [to_np(x) for x in b.get_m()]
    for i in pick:
        pb = oracle_problem(grids[i], hext[i])
        check_terms({t: fields[t][i] for t in TERMS}, pb, m_used[i], "f32", grids[i])
        err = np.abs(got[i] - oracle.rk4(pb, m_used[i], C.dt, 10)).max()
        print(f"grid {i} {grids[i]}: m after 10 steps {err:.2e}")
        assert err <= TRAJ_TOL["f32"], (i, grids[i], err)
