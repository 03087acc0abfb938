"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 path fields <= 1e-11 relative max, FP32 path fields <= 1e-5
relative max (relative to the largest entry of the oracle field), the demag
tensor <= 1e-14 absolute, trajectories after 1000 steps <= 1e-9 (FP64) and
<= 1e-4 (FP32) in m.  FP32 comparisons give the oracle the GPU's own
(FP32-normalised) m so that only the arithmetic differs.
"""
import numpy as np
import pytest

import oracle
from synthetic import SMALL, mT_to_Apm, random_unit_m, smooth_unit_m
from tests.gpu_util import problem, rel_max, to_np

pytestmark = pytest.mark.gpu

mmag = pytest.importorskip("paper_1501_07293_amd")

FIELD_TOL = {"f64": 1e-11, "f32": 1e-5}


def make_sim(pb, precision, **kw):
    return mmag.Sim(pb.nx, pb.ny, pb.nz, pb.cell, Ms=pb.Ms, A=pb.A, Ku=pb.Ku, alpha=pb.alpha,
                    gamma=pb.gamma, precision=precision, demag=pb.demag, **kw)


# ------------------------------------------------------------ tensor (Eqs. 10-11)
@pytest.mark.parametrize("dims", [(1, 1, 1), (4, 3, 2), (9, 5, 3), (32, 8, 1), (17, 30, 4)])
def test_demag_tensor_matches_oracle(dims):
    t = to_np(mmag.demag_tensor(*dims))
    ref = oracle.tensor_table(*dims)
    assert t.shape == ref.shape
    assert np.abs(t - ref).max() <= 1e-14


def wrapped_spectrum(pb, P):
    """Real octant of the DFT of the oracle's tensor in the wrapped padded layout
    (numpy FFT as the library primitive), scaled by 1/(Px Py Pz)."""
    Px, Py, Pz = P
    tab = pb.table()
    out = []
    comps = [0, 1, 2, 3, 4, 5] if Pz > 1 else [0, 1, 3, 5]
    nx, ny, nz = pb.nx, pb.ny, pb.nz
    I = np.arange(-(nx - 1), nx) % Px
    J = np.arange(-(ny - 1), ny) % Py
    K = np.arange(-(nz - 1), nz) % Pz
    for c in comps:
        w = np.zeros((Pz, Py, Px))
        w[np.ix_(K, J, I)] = tab[c]
        f = np.fft.fftn(w) / (Px * Py * Pz)
        oct_ = f[: Pz // 2 + 1, : Py // 2 + 1, : Px // 2 + 1]
        out.append(np.transpose(oct_, (0, 2, 1)))       # stored [kz][kx][ky]
    return np.array(out)


@pytest.mark.parametrize("dims", [(32, 8, 1), (13, 7, 3), (12, 10, 6), (33, 17, 1)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_kernel_spectrum_matches_fft_of_oracle_tensor(dims, precision):
    pb = problem(*dims, cell=5e-9)
    sim = make_sim(pb, precision)
    p = sim.plan()
    spec = to_np(sim.kernel_spectrum())
    ref = wrapped_spectrum(pb, (p["px"], p["py"], p["pz"]))
    # the wrapped tensor is even/odd per axis, so its spectrum is real
    assert np.abs(ref.imag).max() <= 1e-13 * np.abs(ref.real).max()
    assert p["kernel_imag_ratio"] <= 1e-12
    tol = 1e-12 if precision == "f64" else 1e-6
    assert rel_max(spec, ref.real) <= tol


# ---------------------------------------------------- effective-field terms
SHAPES = [(32, 8, 1), (33, 17, 1), (12, 10, 6), (13, 7, 3), (1, 1, 1), (5, 1, 4), (64, 48, 2),
          (100, 36, 3), (1, 40, 2), (70, 3, 5)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_field_terms_match_oracle(dims, precision):
    hext = mT_to_Apm([12.0, -5.0, 3.0])
    pb = problem(*dims, cell=4e-9, Ku=2.0e4, hext=hext)
    m0 = random_unit_m(pb.shape, seed=sum(dims))
    sim = make_sim(pb, precision)
    sim.set_hext(hext)
    sim.set_m(m0)
    m_gpu = to_np(sim.get_m())
    ref = oracle.heff_terms(pb, m_gpu)
    for term in ("exch", "anis", "demag", "ext", "eff"):
        got = to_np(sim.field(term))
        if np.abs(ref[term]).max() == 0:
            assert np.abs(got).max() == 0, term
            continue
        err = rel_max(got, ref[term])
        assert err <= FIELD_TOL[precision], (term, err)


GENERIC_SHAPES = [(32, 8, 1), (12, 10, 6), (64, 48, 2), (64, 64, 16), (33, 17, 3)]


@pytest.mark.parametrize("dims", GENERIC_SHAPES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_generic_and_specialised_passes_agree_with_oracle(dims, precision):
    # The same grid through the size-specialised passes and the runtime-radix ones.
    pb = problem(*dims, cell=3e-9, Ku=1.0e4)
    m0 = random_unit_m(pb.shape, seed=7 + sum(dims))
    ref = None
    for generic in (False, True):
        sim = make_sim(pb, precision, generic_fft=generic)
        sim.set_m(m0)
        m_gpu = to_np(sim.get_m())
        if ref is None:
            ref = oracle.heff_terms(pb, m_gpu)["demag"]
        err = rel_max(to_np(sim.field("demag")), ref)
        assert err <= FIELD_TOL[precision], (generic, err)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_uniform_m_exchange_vanishes_and_cube_demag(precision):
    pb = problem(6, 6, 6, 3e-9)
    m = np.zeros(pb.shape)
    m[0] = 1.0
    sim = make_sim(pb, precision)
    sim.set_m(m)
    assert np.abs(to_np(sim.field("exch"))).max() == 0.0
    hd = to_np(sim.field("demag"))
    # cubic symmetry: the averaged demag factor of a cube is 1/3
    assert abs(hd[0].mean() / pb.Ms + 1.0 / 3.0) < (1e-12 if precision == "f64" else 1e-6)


# --------------------------------------------------------------- trajectories
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_small_config_trajectory(precision):
    c = SMALL
    pb = problem(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma)
    m0 = random_unit_m(pb.shape, seed=0)
    sim = make_sim(pb, precision)
    sim.set_m(m0)
    m_start = to_np(sim.get_m())
    m_ref = oracle.rk4(pb, m_start, c.dt, 1000)
    sim.step(1000, c.dt)
    err1000 = np.abs(to_np(sim.get_m()) - m_ref).max()
    m_ref2 = oracle.rk4(pb, m_ref, c.dt, 1000)
    sim.step(1000, c.dt)
    m2 = to_np(sim.get_m())
    err2000 = np.abs(m2 - m_ref2).max()
    tol = 1e-9 if precision == "f64" else 1e-4
    assert err1000 <= tol, err1000
    assert err2000 <= 10 * tol, err2000
    assert np.abs(np.sqrt((m2 ** 2).sum(axis=0)) - 1).max() < (1e-14 if precision == "f64" else 1e-6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_energy_and_mean_match_oracle(precision):
    hext = mT_to_Apm([-20.0, 3.0, 0.0])
    pb = problem(24, 12, 3, 4e-9, Ku=500.0, hext=hext)
    m0 = smooth_unit_m(pb.shape, seed=3)
    sim = make_sim(pb, precision)
    sim.set_hext(hext)
    sim.set_m(m0)
    m_gpu = to_np(sim.get_m())
    e = sim.energy()
    e_ref = oracle.energy(pb, m_gpu)
    scale = np.abs(e_ref).max()
    tol = 1e-10 if precision == "f64" else 1e-5
    assert np.abs(e - e_ref).max() / scale <= tol, (e, e_ref)
    mm = sim.mean_m()
    assert np.abs(mm - oracle.mean_m(pb, m_gpu)).max() <= (1e-14 if precision == "f64" else 1e-7)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_energy_decreases_under_damping(precision):
    pb = problem(16, 16, 2, 5e-9, Ku=500.0, alpha=0.5, hext=mT_to_Apm([10.0, 0.0, 0.0]))
    sim = make_sim(pb, precision)
    sim.set_hext(pb.hext)
    sim.set_m(random_unit_m(pb.shape, seed=11))
    e_prev = sim.energy()[4]
    for _ in range(30):
        sim.step(5, 1e-13)
        e = sim.energy()[4]
        assert e <= e_prev + (1e-12 if precision == "f64" else 1e-6) * abs(e_prev)
        e_prev = e


def test_graph_replay_matches_eager():
    pb = problem(40, 20, 3, 4e-9, Ku=500.0, alpha=0.3)
    m0 = random_unit_m(pb.shape, seed=5)
    outs = []
    for graph in (False, True):
        sim = make_sim(pb, "f32", graph=graph)
        sim.set_m(m0)
        sim.step(19, 1e-13)     # 2 graph replays of 8 steps + 3 direct steps
        outs.append(to_np(sim.get_m()))
    assert np.array_equal(outs[0], outs[1])


def test_deterministic_bitwise():
    pb = problem(48, 24, 4, 4e-9, Ku=500.0)
    m0 = random_unit_m(pb.shape, seed=6)
    outs = []
    for _ in range(2):
        sim = make_sim(pb, "f32")
        sim.set_m(m0)
        sim.step(10, 1e-13)
        outs.append((to_np(sim.get_m()), sim.energy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("dims", [(32, 8, 1), (13, 7, 3), (24, 12, 3)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_max_torque_matches_oracle(dims, precision):
    hext = mT_to_Apm([-20.0, 3.0, 4.0])
    pb = problem(*dims, cell=4e-9, Ku=2.0e4, hext=hext)
    sim = make_sim(pb, precision)
    sim.set_hext(hext)
    sim.set_m(smooth_unit_m(pb.shape, seed=sum(dims)))
    m_gpu = to_np(sim.get_m())
    got, ref = sim.max_torque(), oracle.max_torque(pb, m_gpu)
    print(f"{dims} {precision}: max |m x H| {got:.9e} oracle {ref:.9e}")
    assert abs(got - ref) <= (1e-11 if precision == "f64" else 1e-5) * ref
    # uniform m along a field that has no other torque: a single cell along H_ext
    one = problem(1, 1, 1, 4e-9, Ku=0.0, hext=(3.0e4, 0.0, 0.0))
    s1 = make_sim(one, precision)
    s1.set_hext(one.hext)
    s1.set_m(np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1))
    assert s1.max_torque() <= 1e-12 * 3.0e4


def relaxed_mid_film(seed=0, max_steps=20000, chunk=500, tol=1e-5):
    """The mid film's relaxed seeded state: seeded random m, alpha 0.5, no field,
    dt 5e-14 s, RK4 in FP64 on the GPU until max |m x H_eff| / Ms < tol or
    max_steps steps.  Returns (m, steps run, final max torque / Ms)."""
    from synthetic import MID
    c = MID
    relax = mmag.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=0.5, gamma=c.gamma,
                     precision="f64", graph=True)
    relax.set_m(random_unit_m(c.shape, seed=seed))
    steps, torque = 0, relax.max_torque() / c.Ms
    while steps < max_steps and torque >= tol:
        relax.step(chunk, c.dt)
        steps += chunk
        torque = relax.max_torque() / c.Ms
    return to_np(relax.get_m()), steps, torque


def test_fp32_vs_fp64_gpu_agree_mid_film():
    # 256x64x4 film: relax a seeded random state (alpha 0.5, no field) until the largest
    # torque falls below 1e-5 Ms or 20000 steps, then apply the step field (-20, 3, 0) mT
    # with alpha 0.02, dt 5e-14 s; FP32 tracks FP64 over 1000 steps.
    from synthetic import MID
    c = MID
    m_relaxed, steps, torque = relaxed_mid_film()
    print(f"mid film relaxed after {steps} steps, max |m x H|/Ms = {torque:.2e}")
    assert torque < 1e-5 or steps >= 20000
    res = []
    for prec in ("f64", "f32"):
        sim = mmag.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha,
                       gamma=c.gamma, precision=prec)
        sim.set_hext(c.hext)
        sim.set_m(m_relaxed)
        sim.step(1000, c.dt)
        res.append(to_np(sim.get_m()))
    err = np.abs(res[0] - res[1]).max()
    print("mid film FP32 vs FP64 after 1000 steps:", err)
    assert err <= 1e-4


def test_autotuner_picks_a_schedule_that_matches_the_oracle():
    # 65x33x3: candidates are 7-smooth (135, 70, 6), power-of-two (256, 128, 8) or fast
    # (160, 96 or 128, 8) padding, specialised or runtime-radix passes, 256 or 512 threads;
    # which one wins is a matter of timing, the field must match the oracle whichever.
    pb = problem(65, 33, 3, 4e-9, Ku=500.0)
    m0 = random_unit_m(pb.shape, seed=17)
    sim = make_sim(pb, "f32", autotune=True)
    p = sim.plan()
    print("autotuner choice:", p)
    assert p["tuned"] == 1 and p["candidates"] >= 8 and p["tuned_demag_ms"] > 0
    assert p["px"] in (135, 160, 256) and p["py"] in (70, 96, 128) and p["pz"] in (6, 8)
    sim.set_m(m0)
    m_gpu = to_np(sim.get_m())
    ref = oracle.heff_terms(pb, m_gpu)["demag"]
    assert rel_max(to_np(sim.field("demag")), ref) <= FIELD_TOL["f32"]
    again = make_sim(pb, "f32", autotune=True)       # served from the cache
    q = again.plan()
    assert q["tuned"] == 1 and q["candidates"] == 0
    assert (q["px"], q["py"], q["pz"], q["generic_fft"]) == (p["px"], p["py"], p["pz"], p["generic_fft"])


@pytest.mark.parametrize("dims", [(8, 8, 8), (13, 6, 1), (10, 7, 3)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_euler_matches_oracle(dims, precision):
    # The paper's explicit Euler + renormalisation on standard-problem-#3-like material
    # (Ms 1000 kA/m, A 1e-11 J/m, H_anis 100 kA/m along x, large damping).
    Ms = 1.0e6
    Ku = 4e-7 * np.pi * Ms * 1.0e5 / 2
    pb = problem(*dims, cell=4e-9, Ms=Ms, A=1e-11, Ku=Ku, alpha=1.0)
    m0 = random_unit_m(pb.shape, seed=31)
    sim = make_sim(pb, precision)
    sim.set_m(m0)
    m_used = to_np(sim.get_m())
    sim.step_euler(25, 2e-14)
    ref = oracle.euler(pb, m_used, 2e-14, 25)
    err = np.abs(to_np(sim.get_m()) - ref).max()
    assert err <= (1e-11 if precision == "f64" else 2e-5), err


def test_euler_graph_replay_matches_eager():
    # 37 Euler steps (four replays of an 8-step graph, then 5 eager steps), twice in a
    # row, against the same steps without the graph: bitwise.
    dims = (24, 10, 2)
    pb = problem(*dims, cell=4e-9, Ku=500.0, alpha=0.5)
    m0 = random_unit_m(pb.shape, seed=33)
    out = []
    for graph in (False, True):
        sim = mmag.Sim(*dims, 4e-9, Ku=500.0, alpha=0.5, precision="f32", graph=graph)
        sim.set_m(m0)
        sim.step_euler(37, 2e-14)
        sim.step(3, 2e-14)          # an RK4 step in between takes the graph slot back
        sim.step_euler(37, 2e-14)
        out.append(to_np(sim.get_m()))
    assert np.array_equal(out[0], out[1])



@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(1024, 4, 1), (8, 1024, 1), (128, 128, 32), (2000, 3, 1)])
def test_largest_lengths_sampled_against_direct_sum(dims, precision):
    # The longest lines of each pass: x and y padded to 2048 (specialised x pass in FP32,
    # runtime-radix y k-space beyond 1024), z padded to 64 (specialised z k-space in
    # FP32), and a 7-smooth x length of 4000.  The demag field at 64 sampled cells plus
    # the corners against the oracle's direct sum on the same m.
    pb = problem(*dims, cell=3e-9)
    sim = make_sim(pb, precision)
    sim.set_m(random_unit_m(pb.shape, seed=61))
    m_gpu = to_np(sim.get_m())
    h = to_np(sim.field("demag")).reshape(3, -1)
    N = pb.N
    g = np.random.default_rng(62)
    obs = np.unique(np.concatenate([[0, pb.nx - 1, N - pb.nx, N - 1], g.integers(0, N, 64)]))
    ref = oracle.demag(pb, m_gpu, obs.astype(np.int64))
    err = rel_max(h[:, obs], ref)
    print(f"{dims} {precision} plan {sim.plan()['px']}x{sim.plan()['py']}x{sim.plan()['pz']}: {err:.2e}")
    assert err <= FIELD_TOL[precision]


def test_cube_256_sampled_against_direct_sum():
    # The largest cube of the Euler sweep: 256^3 cells (standard-problem-#3 material),
    # padded 512^3, so the z k-space pass runs with its length fixed at 512.  Demag and
    # effective field at 160 observation cells (all 8 corners, cells on every edge and
    # face, the rest uniform) against the oracle's direct sum, FP64 then FP32; a few
    # Euler steps keep every cell unit length.
    import synthetic
    n = 256
    Ms = 1.0e6
    pb = problem(n, n, n, cell=34e-9 / n, Ms=Ms, A=1e-11, Ku=4e-7 * np.pi * Ms * 1.0e5 / 2, alpha=1.0)
    obs = synthetic.observation_cells(n, n, n, 160, seed=257)
    m0 = random_unit_m(pb.shape, seed=256)
    for precision in ("f64", "f32"):
        sim = make_sim(pb, precision)
        assert sim.plan()["pz"] == 512
        sim.set_m(m0)
        m_gpu = to_np(sim.get_m())
        hd_ref = oracle.demag(pb, m_gpu, obs)
        err = rel_max(to_np(sim.field("demag")).reshape(3, -1)[:, obs], hd_ref)
        ref = hd_ref + oracle.exchange(pb, m_gpu).reshape(3, -1)[:, obs] + \
            oracle.anisotropy(pb, m_gpu).reshape(3, -1)[:, obs]
        err_eff = rel_max(to_np(sim.field("eff")).reshape(3, -1)[:, obs], ref)
        print(f"256^3 {precision}: demag {err:.2e}, effective {err_eff:.2e}", flush=True)
        assert err <= FIELD_TOL[precision] and err_eff <= FIELD_TOL[precision]
        sim.step_euler(4, 1e-14)
        m = to_np(sim.get_m())
        assert np.abs(np.sqrt((m * m).sum(axis=0)) - 1).max() < (1e-12 if precision == "f64" else 1e-6)
        sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(8, 8, 64), (5, 4, 256), (3, 2, 512)])
def test_long_z_lines_match_oracle(dims, precision):
    # z padded to 128, 512 and 1024: the k-space pass with the length fixed at compile
    # time, against the runtime-radix pass and the oracle's direct sum.
    pb = problem(*dims, cell=3e-9, Ku=1.0e4)
    m0 = random_unit_m(pb.shape, seed=71 + dims[2])
    ref = None
    for generic in (False, True):
        sim = make_sim(pb, precision, generic_fft=generic)
        sim.set_m(m0)
        m_gpu = to_np(sim.get_m())
        if ref is None:
            ref = oracle.heff_terms(pb, m_gpu)["demag"]
        err = rel_max(to_np(sim.field("demag")), ref)
        print(f"{dims} {precision} generic={generic} pz={sim.plan()['pz']}: {err:.2e}")
        assert err <= FIELD_TOL[precision], (generic, err)


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("cfg_name", ["LARGE", "MID"])
def test_full_size_configs_against_direct_sum(cfg_name, precision):
    # The 512x512x16 film (padded 1024x1024x32) and the 256x64x4 film (512x128x8) at full
    # size, in the launch configuration the benchmark times (default options).  The film:
    # demag and effective field at 1024 seeded observation cells (all 8 corners, cells on
    # every edge and face, the rest uniform) against the oracle's direct sum.  The
    # mid-size film: at every one of its 65536 cells.  Five RK4 steps keep |m| = 1.
    import synthetic
    c = getattr(synthetic, cfg_name)
    pb = problem(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                 hext=c.hext)
    sim = make_sim(pb, precision)
    sim.set_hext(c.hext)
    sim.set_m(random_unit_m(pb.shape, seed=101))
    m_gpu = to_np(sim.get_m())
    N = pb.N
    obs = synthetic.observation_cells(c.nx, c.ny, c.nz, 1024, seed=102) if cfg_name == "LARGE" \
        else np.arange(N, dtype=np.int64)
    assert len(obs) >= 1024
    hd_ref = oracle.demag(pb, m_gpu, obs)
    hd = to_np(sim.field("demag")).reshape(3, -1)[:, obs]
    err = rel_max(hd, hd_ref)
    heff = to_np(sim.field("eff")).reshape(3, -1)[:, obs]
    ref = hd_ref + oracle.exchange(pb, m_gpu).reshape(3, -1)[:, obs] + \
        oracle.anisotropy(pb, m_gpu).reshape(3, -1)[:, obs] + np.asarray(c.hext).reshape(3, 1)
    err_eff = rel_max(heff, ref)
    print(f"{cfg_name} {precision} ({len(obs)} cells): demag {err:.2e}, effective {err_eff:.2e}")
    assert err <= FIELD_TOL[precision] and err_eff <= FIELD_TOL[precision]
    sim.step(5, c.dt)
    m = to_np(sim.get_m())
    assert np.abs(np.sqrt((m * m).sum(axis=0)) - 1).max() < (1e-12 if precision == "f64" else 1e-6)
