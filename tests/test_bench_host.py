"""Host logic of bench.py (no GPU): the per-kernel byte model of one RK4 step, the
kernel symbols it names for the library's dispatch, the counter record it reports
as roofline.traffic, and its refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FILM = {"px": 1024, "py": 1024, "pz": 32, "hx": 513, "passes": 5, "threads": 256, "generic_fft": 0,
        "x_lines": 8, "x_lines_inv": 4, "spectrum_elems": 6 * 17 * 513 * 513}
FILM_N = (512, 512, 16)
WORKLOAD = ("large film 512x512x16 cells=4194304 cell=3e-09 m, RK4 dt=5e-14 s, "
            "padded FFT 1024x1024x32")


def test_film_step_moves_1605_bytes_per_cell():
    # per cell of the 512x512x16 film in FP32: x passes 3*4 B of m plus 3 complex
    # values of 8 B for each of 513/512 x bins; y passes those plus 1024/512 y bins;
    # k-space two full-y spectra and the 6 x 17 x 513 x 513 octant; LLG 21/4 vectors
    N = 512 * 512 * 16
    b = bench.algorithmic_bytes(FILM, *FILM_N, 4)
    per = {k: v / N for k, v in b.items()}
    assert per["x_fwd"] == pytest.approx(12 + 24 * 513 / 512)
    assert per["y_fwd"] == pytest.approx(24 * 513 / 512 * 3)
    assert per["kspace"] == pytest.approx(96 * 513 / 512 + 6 * 17 * 513 * 513 * 4 / N)
    assert per["llg"] == pytest.approx(63.0)
    assert b["y_inv"] == b["y_fwd"] and b["x_inv"] == b["x_fwd"]
    assert 4 * sum(b.values()) / N == pytest.approx(1604.65, abs=0.01)


def test_periodic_film_step_moves_759_bytes_per_cell():
    plan = dict(FILM, px=512, py=512, hx=257, spectrum_elems=6 * 17 * 257 * 257)
    N = 512 * 512 * 16
    b = bench.algorithmic_bytes(plan, *FILM_N, 4)
    assert 4 * sum(b.values()) / N == pytest.approx(759.2, abs=0.05)


def test_kernel_symbols_follow_the_dispatch():
    sym = lambda k, p="f32", plan=FILM, n=FILM_N: bench.mm_kernel_symbol(k, p, plan, n)
    assert sym("x_fwd") == "mm::k_xfwd<float, 1024, 8, false>"
    assert sym("x_inv") == "mm::k_xinv<float, 1024, 4, false>"
    assert sym("y_fwd") == "mm::k_yline<float, 1024, false, false>"
    assert sym("y_inv") == "mm::k_yline<float, 1024, true, false>"
    assert sym("kspace") == "mm::k_kspace_z<float, 32>"
    assert sym("llg") == "mm::k_llg_stage<float, 2, 2>"
    # planes per thread of the stage update: 1 or 2 for grids one or two cells thick
    assert sym("llg", n=(512, 512, 1)) == "mm::k_llg_stage<float, 1, 2>"
    assert sym("llg", n=(512, 512, 2)) == "mm::k_llg_stage<float, 2, 2>"
    # rows per work-group tile: 2 where the plane splits into 128 x 2 tiles, else 1
    assert sym("llg", n=(384, 500, 16)) == "mm::k_llg_stage<float, 2, 2>"
    assert sym("llg", n=(500, 512, 16)) == "mm::k_llg_stage<float, 2, 1>"
    assert sym("llg", n=(512, 511, 16)) == "mm::k_llg_stage<float, 2, 1>"
    # small one-cell-thick grids: the fused stage pass; two cells thick: the two-plane pass
    small = dict(FILM, px=256, py=256, pz=1, hx=129, passes=3, fused_stage=1)
    assert sym("llg", plan=small, n=(128, 128, 1)) == "mm::k_fused_stage<float, 256, 1, true>"
    # 3-D: lines by the ny nz rows, within 512 threads
    assert sym("llg", plan=dict(small, pz=128), n=(64, 64, 64)) == "mm::k_fused_stage<float, 256, 4, false>"
    assert sym("llg", plan=dict(small, px=1024, pz=32), n=(512, 128, 16)) == "mm::k_fused_stage<float, 1024, 1, false>"
    assert sym("llg", plan=dict(small, px=160, pz=32), n=(80, 512, 16)) == "mm::k_fused_stage<float, 160, 4, false>"
    # at most 256 work-groups: the prefetching instantiation
    assert sym("llg", plan=dict(small, px=512, pz=8), n=(256, 64, 4)) == "mm::k_fused_stage<float, 512, 1, true>"
    two = dict(FILM, px=128, py=128, pz=4, hx=65, passes=3, two_plane=1)
    assert sym("kspace", plan=two, n=(33, 47, 2)) == "mm::k_kspace_y2<float, 128, false>"
    # FP64 lines with a zero upper half take the two-lane z pass
    assert sym("kspace", "f64") == "mm::k_kspace_z_split<double, 32>"
    # periodic x and y: whole lines
    per = dict(FILM, px=512, py=512, hx=257)
    assert sym("x_fwd", plan=per) == "mm::k_xfwd<float, 512, 8, true>"
    assert sym("y_inv", plan=per) == "mm::k_yline<float, 512, true, true>"
    # runtime-radix passes, longer z lines, one cell thick, the fused y-z pass
    gen = dict(FILM, generic_fft=1)
    assert sym("x_fwd", plan=gen) == "mm::k_row_r2c<float, 256>"
    assert sym("kspace", plan=gen) == "mm::k_kspace<float, 256>"
    cube = dict(FILM, px=256, py=256, pz=256)
    assert sym("kspace", plan=cube, n=(128, 128, 128)) == "mm::k_kspace_zl<float, 256, 16>"
    cube512 = dict(cube, px=512, py=512, pz=512)
    assert sym("kspace", plan=cube512, n=(256, 256, 256)) == "mm::k_kspace_zl<float, 512, 4>"
    assert sym("kspace", "f64", plan=cube512, n=(256, 256, 256)) == "mm::k_kspace_zl<double, 512, 4>"
    # FP64 lines of 1024 points keep the LDS-staged pass
    cube1k = dict(cube, px=1024, py=1024, pz=1024)
    assert sym("kspace", "f64", plan=cube1k, n=(512, 512, 512)) == "mm::k_kspace_fixed<double, 256, 1024>"
    thin = dict(FILM, pz=1, passes=3)
    assert sym("kspace", plan=thin, n=(512, 512, 1)) == "mm::k_kspace_y<float, 1024, false>"
    fused = dict(FILM, px=512, py=128, pz=8, passes=3)
    assert sym("kspace", plan=fused, n=(256, 64, 4)) == "mm::k_kspace_yz<float, 256>"
    one = dict(FILM, px=64, py=16, pz=1, hx=33, passes=1)
    assert sym("kspace", plan=one, n=(32, 8, 1)) == "mm::k_demag_1wg<float, 256>"


def test_one_work_group_model_reads_m_and_octant_once():
    plan = dict(FILM, px=64, py=16, pz=1, hx=33, passes=1, spectrum_elems=4 * 1 * 33 * 9)
    b = bench.algorithmic_bytes(plan, 32, 8, 1, 4)
    assert b["kspace"] == 2 * 3 * 256 * 4 + 4 * 33 * 9 * 4
    assert b["x_fwd"] == b["y_fwd"] == b["y_inv"] == b["x_inv"] == 0


def current_record():
    rec = bench.recorded_traffic("mm::k_kspace_z<float, 32>", WORKLOAD)
    if rec is None:
        pytest.skip("the committed counter record predates the current kernel sources")
    return rec


def test_every_profiled_kernel_has_its_byte_model():
    # the committed summary lists each per-step kernel under the symbol the model names
    rec = current_record()
    assert rec["source"].startswith("profiles/")
    text = open(os.path.join(ROOT, rec["source"])).read()
    for k in ("x_fwd", "y_fwd", "kspace", "y_inv", "x_inv", "llg"):
        assert f"`{bench.mm_kernel_symbol(k, 'f32', FILM, FILM_N)}`" in text, k


def test_traffic_record_is_dropped_when_sources_change(monkeypatch):
    rec = current_record()
    alg = bench.algorithmic_bytes(FILM, *FILM_N, 4)["kspace"]
    assert 0.99 < rec["bytes"] / alg < 1.1
    assert bench.recorded_traffic("mm::k_kspace_z<float, 32>", "another workload") is None
    monkeypatch.setattr(bench, "tu_digest", lambda tu: "0" * 64)
    assert bench.recorded_traffic("mm::k_kspace_z<float, 32>", WORKLOAD) is None


def test_grid_cells_from_plan_or_workload():
    assert bench.grid_cells({"n": [3, 4, 5]}) == (3, 4, 5)
    assert bench.grid_cells({}, WORKLOAD) == FILM_N
    assert bench.grid_cells({}, "no sizes here") is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_algorithmic_bytes_of_the_batched_schedules():
    # the byte model the batched leg sums over its grids, on plans as the library
    # reports them (mm_batch_get_grid_plan).  32x8x1 at 64 x 16 points: 33 x bins,
    # 4 kernel spectra, three passes (one cell thick)
    N = 256
    real3, half_x, kern = 3 * N * 4, 3 * 8 * 33 * 8, 4 * 33 * 9 * 4
    one = (real3 + half_x) * 2 + (2 * half_x + kern) + 21 * 3 * N * 4 // 4
    p1 = {"hx": 33, "py": 16, "passes": 3, "spectrum_elems": 4 * 33 * 9}
    assert sum(bench.algorithmic_bytes(p1, 32, 8, 1, 4).values()) == one
    # 33x47x2 under the two-plane schedule at 128 x 128 points: x passes on
    # [3][2][65][47], one y pass reading and writing that spectrum and the 10
    # coefficient planes of 65 x 65 values
    N2 = 33 * 47 * 2
    real3b, half_xb, kernb = 3 * N2 * 4, 3 * 2 * 47 * 65 * 8, 10 * 65 * 65 * 4
    two = (real3b + half_xb) * 2 + (2 * half_xb + kernb) + 21 * 3 * N2 * 4 // 4
    p2 = {"hx": 65, "py": 128, "passes": 3, "spectrum_elems": 10 * 65 * 65}
    assert sum(bench.algorithmic_bytes(p2, 33, 47, 2, 4).values()) == two
    # the same grid through five passes (z transformed, Pz = 4): the y passes expand
    # to the padded 128 rows and the octant has 6 x 3 planes
    full_y = 3 * 2 * 128 * 65 * 8
    five = (real3b + half_xb) * 2 + 2 * (half_xb + full_y) + (2 * full_y + 6 * 3 * 65 * 65 * 4) \
        + 21 * 3 * N2 * 4 // 4
    p5 = {"hx": 65, "py": 128, "passes": 5, "spectrum_elems": 6 * 3 * 65 * 65}
    assert sum(bench.algorithmic_bytes(p5, 33, 47, 2, 4).values()) == five
    assert two < five / 2
