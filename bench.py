"""Throughput of the micromagnetic RK4 step on one MI355X.

Workload (default): the 512 x 512 x 16 film (4.19M cubic cells of 3 nm,
Ms 8e5 A/m, A 1.3e-11 J/m, Ku 0, alpha 0.1, H_ext 0, seeded random m), FP32,
zero-padded FFT 1024 x 1024 x 32, RK4 dt 5e-14 s.  A step is one full RK4 step:
four effective-field evaluations (five FFT passes each) and four fused
LLG/RK4 stage passes.  value = cells * steps / seconds (cell-updates/s).

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (its average launch time measured with HIP events inside the timed
region), an FP64 leg, the sampled field error against the FP64 oracle, and the
oracle timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_EVERY = 8       # launches of the dominant kernel per timed launch in the timed region
KERNEL_IDS = ["x_fwd", "y_fwd", "kspace", "y_inv", "x_inv", "llg"]
PROFILES = os.path.join(ROOT, "profiles")
# counter readings of a plain 1 GiB device copy (1 GiB read, 1 GiB written) under
# rocprofv3 --pmc on MI355X: FETCH_SIZE reads 524299.5 KiB, WRITE_SIZE 1048576 KiB
COPY_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}


CSRC = os.path.join(ROOT, "paper_1501_07293_amd", "csrc")
# translation unit that defines each kernel family
KERNEL_TU = [("mm::kbf_", "mm_batch.hip"), ("mm::kb_", "mm_batch.hip"),
             ("mm::k_xfwd", "mm_fast.hip"), ("mm::k_xinv", "mm_fast.hip"),
             ("mm::k_yline", "mm_fast.hip"), ("mm::k_kspace_z", "mm_fast.hip"),
             ("mm::k_kspace_y", "mm_fast.hip"), ("mm::k_fused_", "mm_fused.hip"),
             ("mm::k_llg_stage", "mm_llg.hip"),
             ("mm::k_row_", "mm_passes.hip"), ("mm::k_col_fft", "mm_passes.hip"),
             ("mm::k_kspace<", "mm_passes.hip"), ("mm::k_kspace_fixed", "mm_passes.hip")]


def tu_digest(tu: str) -> str:
    """sha256 over a translation unit, the headers it includes (transitively) and
    the build flags, so that counter readings taken on one build of a kernel are
    not reported for another."""
    import hashlib
    import re
    seen, todo = [], [tu]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.append(f)
        todo += re.findall(r'#include "(mm_[a-z_]+\.hpp)"', open(os.path.join(CSRC, f)).read())
    h = hashlib.sha256()
    for f in sorted(seen) + ["../build.py"]:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_digest(kernel: str) -> str | None:
    for prefix, tu in KERNEL_TU:
        if kernel.startswith(prefix):
            return tu_digest(tu)
    return None


def recorded_traffic(kernel: str, workload: str) -> dict | None:
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summaries (FETCH_SIZE and WRITE_SIZE, each scaled by the copy calibration);
    None when no summary covers it or its sources changed since it was taken."""
    if not os.path.isdir(PROFILES):
        return None
    digest = kernel_digest(kernel)
    for f in sorted(os.listdir(PROFILES)):
        if not f.endswith(".md"):
            continue
        text = open(os.path.join(PROFILES, f)).read()
        start = text.find("```json\n")
        if start < 0:
            continue
        end = text.find("```", start + 8)
        try:
            rec = json.loads(text[start + 8:end])
        except ValueError:
            continue
        if rec.get("workload") != workload:
            continue
        k = rec.get("kernels", {}).get(kernel)
        if k and k.get("hbm_bytes_per_launch") and digest and k.get("sources_sha256") == digest:
            return {"bytes": k["hbm_bytes_per_launch"], "source": f"profiles/{f}",
                    "avg_ns": k.get("avg_ns")}
    return None


def algorithmic_bytes(plan: dict, nx: int, ny: int, nz: int, esz: int) -> dict:
    """Bytes each kernel must move per launch (reads + writes of its inputs and
    outputs once, nothing for the zero padding it never stores)."""
    N = nx * ny * nz
    hx, Py = plan["hx"], plan["py"]
    cz = 2 * esz                           # one complex value
    real3 = 3 * N * esz                    # m or H, three components
    half_x = 3 * nz * ny * hx * cz         # after the x pass
    if plan["passes"] == 1:                # one work-group: m in, field out, octant
        b = {"x_fwd": 0, "y_fwd": 0, "kspace": 2 * real3 + plan["spectrum_elems"] * esz, "y_inv": 0,
             "x_inv": 0}
    elif plan["passes"] == 5:
        full_y = 3 * nz * Py * hx * cz     # after the y pass
        kern = plan["spectrum_elems"] * esz
        b = {"x_fwd": real3 + half_x, "y_fwd": half_x + full_y, "kspace": 2 * full_y + kern,
             "y_inv": full_y + half_x, "x_inv": half_x + real3}
    else:
        kern = plan["spectrum_elems"] * esz
        b = {"x_fwd": real3 + half_x, "y_fwd": 0, "kspace": 2 * half_x + kern, "y_inv": 0,
             "x_inv": half_x + real3}
    # LLG stage: reads m_s, H_d (+ m_n, acc for stages 2-4), writes acc/out:
    # 4, 6, 6, 5 vector arrays -> 21/4 vector arrays on average per launch.
    b["llg"] = int(21 * 3 * N * esz / 4)
    return b


def run_gpu(args, cfg, precision: str, steps: int, warmup: int, profile: bool, repeats: int = 1,
            autotune: bool = False, graph: bool | None = None):
    """Times `repeats` runs of exactly `steps` RK4 steps (each bracketed by device
    synchronisation) after `warmup` untimed steps; returns the handle, its plan,
    the list of run times, the per-kernel averages of a short untimed profiling
    pass, and the dominant kernel's average launch time over all timed runs
    (HIP events around one launch in PROFILE_EVERY).  graph: replay step graphs
    (default: the --graph flag)."""
    import torch

    import paper_1501_07293_amd as mm
    from synthetic import random_unit_m

    sim = mm.Sim(cfg.nx, cfg.ny, cfg.nz, cfg.cell, Ms=cfg.Ms, A=cfg.A, Ku=cfg.Ku, alpha=cfg.alpha,
                 gamma=cfg.gamma, precision=precision, graph=args.graph if graph is None else graph,
                 autotune=autotune, device="cuda:0")
    sim.set_hext(cfg.hext)
    m0 = random_unit_m(cfg.shape, seed=0)
    sim.set_m(m0)
    plan = sim.plan()
    sim.step(warmup, cfg.dt)
    torch.cuda.synchronize()
    per_kernel = {}
    if profile:
        # short untimed pass: average duration of every kernel class
        for k in KERNEL_IDS:
            if plan["passes"] == 3 and k in ("y_fwd", "y_inv"):
                continue
            sim.profile_begin(k)
            sim.step(2, cfg.dt)
            ms, n = sim.profile_end()
            per_kernel[k] = (ms / max(n, 1), n)
        dom = max(per_kernel, key=lambda k: per_kernel[k][0] * per_kernel[k][1])
        # the timed region brackets one launch in PROFILE_EVERY of the dominant
        # kernel with HIP events (an event pair on every launch costs ~1.6% of the step)
        sim.profile_begin(dom, every=PROFILE_EVERY)
    else:
        dom = None
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps, cfg.dt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dom_ms = dom_n = None
    if dom is not None:
        tot, dom_n = sim.profile_end()
        dom_ms = tot / max(dom_n, 1)
    energy = sim.energy()
    return sim, plan, times, per_kernel, dom, dom_ms, dom_n, energy


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 20) -> float:
    """GB/s of a plain device-to-device copy (read + write counted) on this GPU."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes * reps / dt / 1e9


def batched_leg(steps: int, autotune: bool, warmup: int = 2, check: bool = False,
                repeats: int = 5, layout: str = "7smooth") -> dict:
    """512 uneven grids (nx, ny in [32, 128], nz in {1, 2}), FP32, one launch per pass
    over all grids, graph replay; value = total cells * steps / s.  autotune: the
    layout (padding and pass family) is timed at creation; otherwise `layout`:
    "7smooth" (7-smooth padding, runtime-radix passes), "pow2" (power-of-two padding,
    size-class passes) or "fast" (powers of two and 96, 160, 192, 224, size-class
    passes)."""
    import torch

    import paper_1501_07293_amd as mm
    import synthetic
    c = synthetic.BATCH_TEMPLATE
    samples = synthetic.batch_samples(512, seed=0)
    grids = [(s.nx, s.ny, s.nz) for s in samples]
    hext = np.array([s.hext for s in samples])
    b = mm.BatchSim(grids, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                    hext=hext, precision="f32", graph=True, autotune=autotune,
                    pow2_pad=not autotune and layout == "pow2",
                    fast_pad=not autotune and layout == "fast")
    info = b.info()
    b.set_m([synthetic.random_unit_m((3, s.nz, s.ny, s.nx), seed=s.seed) for s in samples])
    b.step(warmup, c.dt)
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps, c.dt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    pad = "pow2" if info["pow2_pad"] else ("fast" if info["fast_pad"] else "7-smooth")
    # the padded sizes and schedule each grid runs with (size classes may pad a grid
    # beyond its own automatic length)
    step_bytes = sum(4 * sum(algorithmic_bytes(b.grid_plan(i), nx, ny, nz, 4).values())
                     for i, (nx, ny, nz) in enumerate(grids))
    out = {"grids": len(grids), "cells": b.cells, "steps": steps, "ms_per_step": 1e3 * dt / steps,
           "value": b.cells * steps / dt, "unit": "cell-updates/s", "dtype": "f32",
           "step_model_bytes": step_bytes, "effective_gbs": step_bytes / (dt / steps) / 1e9,
           "padding": {"pow2": "power of two", "fast": "powers of two and 96, 160, 192, 224",
                       "7-smooth": "7-smooth"}[pad],
           "step_model_bytes_per_cell": step_bytes / b.cells,
           "passes": "size classes" if info["size_classes"] else "runtime radix",
           "autotuned": bool(info["tuned"]), "layouts_timed": info["candidates"],
           "repeats": len(times)}
    if check:
        out["err"] = batch_oracle_error(b, grids, hext)
    b.close()
    return out


def periodic_leg(steps: int, warmup: int = 3) -> dict:
    """The 512x512x16 film with periodic x and y (no zero padding: FFT 512x512x32),
    FP32, RK4: whole-job rate, per-kernel launch times and their algorithmic
    bandwidth."""
    import torch

    import paper_1501_07293_amd as mm
    import synthetic
    c = synthetic.LARGE
    sim = mm.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                 precision="f32", periodic=(True, True, False), device="cuda:0")
    sim.set_hext(c.hext)
    sim.set_m(synthetic.random_unit_m(c.shape, seed=0))
    plan = sim.plan()
    sim.step(warmup, c.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, c.dt)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ab = algorithmic_bytes(plan, c.nx, c.ny, c.nz, 4)
    kernels = {}
    for k in KERNEL_IDS:
        sim.profile_begin(k)
        sim.step(2, c.dt)
        ms, n = sim.profile_end()
        if n:
            kernels[k] = {"avg_us": 1e3 * ms / n, "gbs": ab[k] / (ms / n * 1e-3) / 1e9}
    sim.close()
    return {"workload": f"large film {c.nx}x{c.ny}x{c.nz} periodic in x and y, RK4 dt={c.dt} s, "
                        f"FFT {plan['px']}x{plan['py']}x{plan['pz']}",
            "steps": steps, "ms_per_step": 1e3 * secs / steps, "value": c.N * steps / secs,
            "unit": "cell-updates/s", "dtype": "f32", "kernels": kernels,
            "step_model_bytes_per_cell": 4 * sum(ab.values()) / c.N}


def adjoint_leg(check: bool = True, directions: int = 32) -> dict:
    """128x128x1 Ku-map rollout of 500 RK4 steps (checkpoint every 50) and its
    hand-written adjoint, FP32: forward and backward wall time (median of 5), and
    the gradient's error: over seeded Gaussian directions v of the Ku map, the rms
    of (<grad, v> - fd) / rms_projection, fd the Richardson-extrapolated central
    difference of the FP64 forward along v, rms_projection = |grad|_2 |v|_2 / sqrt(N)."""
    import torch

    import paper_1501_07293_amd as mm
    import synthetic
    c = synthetic.DIFF
    sim = mm.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=0.0, alpha=c.alpha, gamma=c.gamma,
                 precision="f32", graph=True)
    ku_np = synthetic.ku_map(c, seed=1)
    m0_np = synthetic.random_unit_m(c.shape, seed=2)
    tgt_np = synthetic.vortex_target(c, seed=3)
    ku = torch.tensor(ku_np, dtype=torch.float32, device="cuda:0", requires_grad=True)
    m0 = torch.tensor(m0_np, dtype=torch.float32, device="cuda:0")
    tgt = torch.tensor(tgt_np, dtype=torch.float32, device="cuda:0")
    # warm-up of both directions at the timed shape (workspace allocations, graphs)
    ((mm.rollout(sim, ku, m0, c.steps, c.dt, 50) - tgt) ** 2).sum(dim=0).mean().backward()
    torch.cuda.synchronize()
    fwd, bwd = [], []
    for _ in range(5):
        ku.grad = None
        t0 = time.perf_counter()
        mf = mm.rollout(sim, ku, m0, c.steps, c.dt, 50)
        loss = ((mf - tgt) ** 2).sum(dim=0).mean()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd.append(t1 - t0)
        bwd.append(t2 - t1)
    grad = ku.grad.double().cpu().numpy()
    sim.close()
    f, b = float(np.median(fwd)), float(np.median(bwd))
    out = {"workload": "128x128x1 Ku-map rollout, 500 RK4 steps, checkpoint 50, FP32 (median of 5)",
           "forward_s": f, "backward_s": b, "backward_over_forward": b / f,
           "forward_us_per_step": 1e6 * f / c.steps,
           "forward_cell_updates_per_s": c.N * c.steps / f}
    if check:
        s64 = mm.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=0.0, alpha=c.alpha, gamma=c.gamma,
                     precision="f64", graph=True)

        def loss64(kmap):
            s64.set_ku_map(kmap)
            s64.set_m(m0_np)
            s64.step(c.steps, c.dt)
            m = s64.get_m().cpu().numpy()
            return float(((m - tgt_np) ** 2).sum(axis=0).mean())

        g = np.random.default_rng(40)
        ratios = []
        for _ in range(directions):
            v = g.standard_normal(ku_np.shape)
            d1 = (loss64(ku_np + 2.0 * v) - loss64(ku_np - 2.0 * v)) / 4.0
            d2 = (loss64(ku_np + 1.0 * v) - loss64(ku_np - 1.0 * v)) / 2.0
            fd = (4 * d2 - d1) / 3
            rms = np.sqrt((grad ** 2).sum()) * np.sqrt((v ** 2).sum() / v.size)
            ratios.append((float((grad * v).sum()) - fd) / rms)
        s64.close()
        out["err"] = {"grad_rel_rms_vs_fd": float(np.sqrt(np.mean(np.square(ratios)))),
                      "directions": directions, "tolerance": 1e-4,
                      "definition": "rms over Gaussian directions v of (<grad,v> - fd)/(|grad| |v| / sqrt(N)); "
                                    "fd: Richardson-extrapolated central differences (eps 2 and 1 J/m^3) of "
                                    "the FP64 GPU forward"}
    return out


PAPER_TABLE1_MS = {8: (3.99, 24.15, 22.58), 16: (26.56, 26.97, 23.97), 32: (248.8, 45.21, 26.89),
                   64: (2903.0, 238.0, 76.24)}   # CPU, GPU FP64, GPU FP32 ms per Euler step


def cube_sweep_leg(steps: int = 200) -> dict:
    """The paper's own benchmark shape: N^3 cubes (standard problem #3 material: Ms 1000 kA/m,
    A 1e-11 J/m, H_anis 100 kA/m, large damping), explicit Euler + renormalisation, ms per
    step in FP32 and FP64; the paper's GTX 650 Ti / Xeon E5410 numbers beside them."""
    import torch

    import paper_1501_07293_amd as mm
    from synthetic import random_unit_m
    Ms = 1.0e6
    Ku = 4e-7 * np.pi * Ms * 1.0e5 / 2
    rows = []
    for n in (8, 16, 32, 64, 128, 256):
        k = steps if n < 256 else max(steps // 4, 8)   # 256^3: milliseconds per step
        row = {"N": n, "steps": k}
        for prec in ("f32", "f64"):
            sim = mm.Sim(n, n, n, 34e-9 / n, Ms=Ms, A=1e-11, Ku=Ku, alpha=1.0, precision=prec,
                         graph=True)
            sim.set_m(random_unit_m((3, n, n, n), seed=n))
            sim.step_euler(16, 1e-14)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step_euler(k, 1e-14)
            torch.cuda.synchronize()
            row[f"ms_per_step_{prec}"] = 1e3 * (time.perf_counter() - t0) / k
            sim.close()
        if n in PAPER_TABLE1_MS:
            cpu, g64, g32 = PAPER_TABLE1_MS[n]
            row["paper_ms_cpu_fp64_fp32"] = [cpu, g64, g32]
        rows.append(row)
    return {"workload": "N^3 cube, explicit Euler + renormalisation, graph replay of 8-step "
                        "groups (context: paper Table 1, other hardware, MATLAB)", "rows": rows}


def sp4_leg() -> dict:
    """The appendix run of the paper (standard problem #4, field 1): 166x42x1 cells of 3 nm,
    150000 explicit Euler steps of 5 fs through the saturate / ramp / relax / reverse
    protocol, <m> every 1000 steps; wall time of the whole protocol in FP32 and FP64."""
    import torch

    import paper_1501_07293_amd as mm
    import synthetic
    c = synthetic.SP4
    out = {"workload": "standard problem 4 protocol, 166x42x1, 150000 Euler steps (appendix script)"}
    for prec in ("f32", "f64"):
        sim = mm.Sim(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha,
                     gamma=c.gamma, precision=prec, graph=True, autotune=True)
        out[f"plan_{prec}"] = {k: sim.plan()[k] for k in ("px", "py", "generic_fft", "x_lines")}
        m0 = np.zeros(c.shape)
        m0[0] = 1.0
        sim.set_m(m0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = sim.run_schedule(synthetic.sp4_pieces(), c.dt, 1000, method="euler")
        torch.cuda.synchronize()
        out[f"seconds_{prec}"] = time.perf_counter() - t0
        t = tr.cpu().numpy()
        out[f"s_state_m_{prec}"] = t[49, 1:].tolist()
        out[f"final_m_{prec}"] = t[-1, 1:].tolist()
        sim.close()
    out["us_per_step_f32"] = 1e6 * out["seconds_f32"] / c.steps
    return out


def field_error_sampled(sim, cfg, pb, nsamp: int, seed: int = 1, every_cell: bool = False):
    """Relative max error of the demag field against the oracle's direct sum at
    `nsamp` seeded observation cells (all corners, cells on every edge and face,
    the rest uniform), or at every cell."""
    import oracle
    from synthetic import observation_cells
    obs = np.arange(cfg.N, dtype=np.int64) if every_cell else \
        observation_cells(cfg.nx, cfg.ny, cfg.nz, nsamp, seed=seed)
    m = sim.get_m().double().cpu().numpy()
    hd = sim.field("demag").double().cpu().numpy().reshape(3, -1)[:, obs]
    t0 = time.perf_counter()
    ref = oracle.demag(pb, m, obs)
    dt = time.perf_counter() - t0
    err = float(np.abs(hd - ref).max() / np.abs(ref).max())
    return err, len(obs), dt, m


def cpu_baseline(cfg, pb, m, target_s: float):
    """The FP64 oracle on the host cores: direct-sum demag on a sample of
    observation cells plus the O(N) local terms over the whole grid, scaled to
    one RK4 step (four field evaluations for every cell)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(7)
    N = cfg.N
    nobs = 16
    t_obs = 0.0
    while True:
        obs = rng.integers(0, N, size=nobs).astype(np.int64)
        t0 = time.perf_counter()
        oracle.demag(pb, m, obs)
        t_obs = time.perf_counter() - t0
        if t_obs > 0.25 * target_s or nobs >= N:
            break
        nobs = int(min(N, nobs * max(2.0, 0.3 * target_s / max(t_obs, 1e-3))))
    t0 = time.perf_counter()
    h = oracle.exchange(pb, m)
    oracle.llg_rhs(pb, m, h)
    t_local = time.perf_counter() - t0
    per_step = 4 * (t_obs / nobs * N + t_local)
    return {"value": N / per_step, "unit": "cell-updates/s", "cores": threads, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"direct-sum demag at {nobs} sampled observation cells ({t_obs:.1f} s) + "
                      f"local terms on all {N} cells ({t_local:.2f} s), scaled to 4 field "
                      f"evaluations per cell per RK4 step (extrapolated; O(N^2) oracle vs "
                      f"O(N log N) GPU path)"}


def mid_leg(args, steps: int) -> dict:
    """The 256x64x4 film (padded 512x128x8) in FP32 with the autotuned schedule (which
    also times the fused y-z pass there) and step-graph replay (its kernels run a few
    microseconds each, so launches cost measurably: 0.0900 against 0.0870 ms per step):
    median rate of 5 runs of `steps` steps and the demag field against the oracle's
    direct sum at every cell."""
    import oracle
    import synthetic
    c = synthetic.MID
    sim, plan, times, _, _, _, _, _ = run_gpu(args, c, "f32", steps, 5, False, repeats=5, autotune=True,
                                              graph=True)
    med = float(np.median(times))
    pb = oracle.Problem(c.nx, c.ny, c.nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha,
                        gamma=c.gamma, hext=tuple(c.hext))
    err, nobs, _, _ = field_error_sampled(sim, c, pb, 0, every_cell=True)
    sim.close()
    return {"workload": f"{c.name} cells={c.N} cell={c.cell:g} m, RK4 dt={c.dt:g} s, "
                        f"padded FFT {plan['px']}x{plan['py']}x{plan['pz']}",
            "steps": steps, "repeats": len(times), "ms_per_step": 1e3 * med / steps,
            "value": c.N * steps / med, "unit": "cell-updates/s", "dtype": "f32", "graph": True,
            "schedule": {k: plan[k] for k in ("passes", "generic_fft", "threads", "tuned", "candidates")},
            "err": {"demag_field_rel_max": err, "cells": nobs, "tolerance": 1e-5}}


def batch_oracle_error(b, grids, hext) -> dict:
    """Fields of 8 grids of a batch (the smallest, the largest, six with odd prime
    nx and ny) against the oracle at every cell: relative max per term, worst."""
    import oracle
    import synthetic
    c = synthetic.BATCH_TEMPLATE

    def isprime(n):
        return n > 2 and all(n % p for p in range(2, int(n ** 0.5) + 1))
    sizes = [g[0] * g[1] * g[2] for g in grids]
    primes = [i for i, g in enumerate(grids) if isprime(g[0]) and isprime(g[1])][:6]
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes))] + primes
    m = [x.double().cpu().numpy() for x in b.get_m()]
    h = [x.double().cpu().numpy() for x in b.field("eff")]
    worst = 0.0
    for i in pick:
        nx, ny, nz = grids[i]
        pb = oracle.Problem(nx, ny, nz, c.cell, Ms=c.Ms, A=c.A, Ku=c.Ku, alpha=c.alpha, gamma=c.gamma,
                            hext=tuple(hext[i]))
        ref = oracle.heff_terms(pb, m[i])["eff"]
        worst = max(worst, float(np.abs(h[i] - ref).max() / np.abs(ref).max()))
    return {"effective_field_rel_max": worst, "grids_checked": pick, "tolerance": 1e-5}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="large", choices=["large", "mid", "small"])
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batched-leg", action="store_true")
    ap.add_argument("--no-adjoint-leg", action="store_true")
    ap.add_argument("--no-cube-leg", action="store_true")
    ap.add_argument("--no-sp4-leg", action="store_true")
    ap.add_argument("--no-periodic-leg", action="store_true")
    ap.add_argument("--no-mid-leg", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--samples", type=int, default=1024)
    ap.add_argument("--leg", default=None, choices=["batched", "adjoint", "mid"],
                    help="run only this leg (FP32) and print its JSON record; for profiling")
    ap.add_argument("--batch-layout", default="auto", choices=["auto", "7smooth", "pow2", "fast"],
                    help="--leg batched: autotuned layout, or a fixed one")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the micromagnetic step runs on one GPU only (got --gpus {args.gpus}); "
              f"sharding a grid or a batch across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic

    if args.leg is not None:
        # one leg alone (no headline run): what a profiler wraps to see that leg's kernels
        if args.leg == "batched":
            rec = batched_leg(args.steps, autotune=args.batch_layout == "auto", warmup=args.warmup,
                              check=not args.no_cpu_baseline, repeats=args.repeats,
                              layout=args.batch_layout)
        elif args.leg == "adjoint":
            rec = adjoint_leg(check=not args.no_cpu_baseline)
        else:
            rec = mid_leg(args, args.steps)
        print(json.dumps({"leg": args.leg, **rec}), flush=True)
        return

    cfg = {"large": synthetic.LARGE, "mid": synthetic.MID, "small": synthetic.SMALL}[args.workload]
    esz = 4 if args.precision == "f32" else 8
    sim, plan, times, per_kernel, dom, dom_ms, dom_n, energy = run_gpu(
        args, cfg, args.precision, args.steps, args.warmup, not args.no_profile, repeats=args.repeats)
    secs = float(np.median(times))
    value = cfg.N * args.steps / secs
    out = {
        "metric": "cell-updates/s per LLG step (FP32 vs FP64 at stated err), % HBM roofline",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"{cfg.name} cells={cfg.N} cell={cfg.cell:g} m, RK4 dt={cfg.dt:g} s, "
                               f"padded FFT {plan['px']}x{plan['py']}x{plan['pz']}",
                   "precision": args.precision, "graph": bool(args.graph),
                   "fft_passes_per_field": plan["passes"], "threads_per_fft_wg": plan["threads"]},
        "timing": {"repeats": len(times), "statistic": "median",
                   "ms_per_step_each": [1e3 * t / args.steps for t in times]},
    }
    if dom is not None:
        ab = algorithmic_bytes(plan, cfg.nx, cfg.ny, cfg.nz, esz)
        achieved = ab[dom] / (dom_ms * 1e-3) / 1e9
        kname = mm_kernel_symbol(dom, args.precision, plan, (cfg.nx, cfg.ny, cfg.nz))
        out["roofline"] = {"bound": "hbm", "kernel": kname,
                           "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "algorithmic_bytes_per_launch": ab[dom], "avg_launch_ms": dom_ms,
                           "launches_timed": dom_n,
                           "frac_source": f"avg_launch_ms: HIP events on the kernel's stream around one "
                                          f"launch in {PROFILE_EVERY} of it during the timed runs"}
        tr = recorded_traffic(kname, out["config"]["workload"])
        if tr is not None:
            # HBM bytes one launch moves (counters), against the algorithmic bytes above
            out["roofline"]["traffic"] = tr["bytes"]
            out["roofline"]["traffic_unit"] = "bytes/launch"
            out["roofline"]["traffic_over_algorithmic"] = tr["bytes"] / ab[dom]
            out["roofline"]["traffic_source"] = tr["source"]
            if tr.get("avg_ns"):
                # the committed rocprofv3 kernel trace of the same kernel and sources
                out["roofline"]["rocprof_avg_launch_ms"] = tr["avg_ns"] * 1e-6
                out["roofline"]["frac_rocprof"] = ab[dom] / (tr["avg_ns"] * 1e-9) / 1e9 / HBM_PEAK_GBS
        step_bytes = 4 * sum(ab.values())
        out["kernels"] = {k: {"avg_ms": v[0], "gbs": ab[k] / (v[0] * 1e-3) / 1e9 if v[0] else None}
                          for k, v in per_kernel.items()}
        out["step_model_bytes_per_cell"] = step_bytes / cfg.N
        out["algorithmic_bytes"] = ab
        out["plan"] = {k: plan[k] for k in ("px", "py", "pz", "passes", "threads", "generic_fft", "x_lines",
                                            "x_lines_inv")}
        out["plan"]["n"] = [cfg.nx, cfg.ny, cfg.nz]
        out["effective_gbs"] = step_bytes / (secs / args.steps) / 1e9
    out["sources_sha256"] = {tu: tu_digest(tu) for tu in sorted({t for _, t in KERNEL_TU})}
    out["energy_J"] = energy.tolist()
    out["copy_gbs_measured"] = copy_bandwidth()

    pb = None
    if not args.no_cpu_baseline:
        import oracle
        pb = oracle.Problem(cfg.nx, cfg.ny, cfg.nz, cfg.cell, Ms=cfg.Ms, A=cfg.A, Ku=cfg.Ku,
                            alpha=cfg.alpha, gamma=cfg.gamma, hext=tuple(cfg.hext))
        t0 = time.perf_counter()
        pb.table()
        t_table = time.perf_counter() - t0
        err, nobs, _, m = field_error_sampled(sim, cfg, pb, args.samples)
        out["err"] = {"demag_field_rel_max_sampled": err, "sampled_cells": nobs,
                      "cells": "all 8 corners, 4 per edge, 16 per face, the rest uniform (seeded)",
                      "tolerance": 1e-5 if args.precision == "f32" else 1e-11}
        cb = cpu_baseline(cfg, pb, m, args.cpu_seconds)
        cb["setup_s"] = t_table
        out["cpu_baseline"] = cb
    sim.close()
    del sim
    torch.cuda.empty_cache()

    if not args.no_fp64_leg and args.precision == "f32":
        fsteps = max(20, args.steps // 10)
        sim64, _, t64, _, _, _, _, _ = run_gpu(args, cfg, "f64", fsteps, 2, False, repeats=args.repeats)
        s64 = float(np.median(t64))
        out["fp64"] = {"value": cfg.N * fsteps / s64, "steps": fsteps, "repeats": len(t64),
                       "ms_per_step": 1e3 * s64 / fsteps}
        if pb is not None:
            e64, n64, _, _ = field_error_sampled(sim64, cfg, pb, args.samples)
            out["fp64"]["err"] = {"demag_field_rel_max_sampled": e64, "sampled_cells": n64,
                                  "tolerance": 1e-11}
        sim64.close()
        del sim64
        torch.cuda.empty_cache()
    if not args.no_mid_leg and args.workload == "large":
        out["mid"] = mid_leg(args, max(50, args.steps))
        torch.cuda.empty_cache()
    if not args.no_batched_leg:
        out["batched"] = batched_leg(max(10, args.steps // 10), autotune=True,
                                     check=not args.no_cpu_baseline)
        out["batched_7smooth"] = batched_leg(max(10, args.steps // 10), autotune=False)
    if not args.no_adjoint_leg:
        out["adjoint"] = adjoint_leg(check=not args.no_cpu_baseline)
    if not args.no_cube_leg:
        out["paper_table1_shape"] = cube_sweep_leg()
    if not args.no_periodic_leg:
        out["periodic"] = periodic_leg(max(10, args.steps // 5))
    if not args.no_sp4_leg:
        out["paper_appendix_sp4"] = sp4_leg()
    print(json.dumps(out), flush=True)


def grid_cells(plan: dict, workload: str = "") -> tuple | None:
    """(nx, ny, nz) from the plan, else from a workload name ('... NXxNYxNZ cells=...')."""
    if plan.get("n"):
        return tuple(plan["n"])
    import re
    mt = re.search(r"(\d+)x(\d+)x(\d+) cells", workload)
    return tuple(int(v) for v in mt.groups()) if mt else None


def mm_kernel_symbol(k: str, precision: str, plan: dict, n: tuple | None = None) -> str:
    """Symbol of the kernel the library launches for pass k under this plan (the
    size-specialised one where it exists, as the library's dispatch decides).
    n = (nx, ny, nz): an axis whose cells fill more than half its FFT length (a
    periodic axis) takes the whole-line instantiation; without n none is assumed."""
    t = "float" if precision == "f32" else "double"
    fast = not plan.get("generic_fft", 0)
    px, py, pz = plan["px"], plan["py"], plan["pz"]
    nx, ny, nz = n if n else (0, 0, 0)
    pow2 = lambda v: v & (v - 1) == 0
    b = lambda v: "true" if v else "false"
    x_ok = fast and pow2(px) and 16 <= px <= (2048 if t == "float" else 1024)
    y_ok = fast and pow2(py) and 16 <= py <= 2048
    if k == "llg":
        if plan.get("fused_stage"):
            # the fused stage pass's row pairs per work-group, as the library picks them:
            # by the ny nz rows, one line from 512 points, at most 512 threads (3 lines of
            # P / R0 threads each)
            rows = ny * nz
            lines = 1 if px >= 512 else (4 if rows >= 2048 else (2 if rows >= 1024 else 1))
            tl = px // {16: 16, 32: 8, 64: 8, 128: 16, 256: 16, 512: 8, 1024: 16}.get(px, 16)
            while lines > 1 and 3 * lines * tl > 512:
                lines //= 2
            # launches of at most 256 work-groups take the prefetching instantiation
            pre = nz * ((ny + 2 * lines - 1) // (2 * lines)) <= 256
            return f"mm::k_fused_stage<{t}, {px}, {lines}, {b(pre)}>"
        kz = 1 if nz == 1 else 2   # planes per thread
        ty = 2 if nx % 128 == 0 and ny % 2 == 0 else 1   # rows per work-group tile
        return f"mm::k_llg_stage<{t}, {kz}, {ty}>"
    if plan["passes"] == 1:
        return f"mm::k_demag_1wg<{t}, {plan['threads']}>"
    if k in ("x_fwd", "x_inv"):
        lines = plan.get("x_lines", 8) if k == "x_fwd" else plan.get("x_lines_inv", 4)
        return f"mm::k_{'xfwd' if k == 'x_fwd' else 'xinv'}<{t}, {px}, {lines}, {b(2 * nx > px)}>" \
            if x_ok else \
            f"mm::k_row_{'r2c' if k == 'x_fwd' else 'c2r'}<{t}, {plan['threads']}>"
    if k in ("y_fwd", "y_inv"):
        return f"mm::k_yline<{t}, {py}, {b(k == 'y_inv')}, {b(2 * ny > py)}>" if y_ok else \
            f"mm::k_col_fft<{t}, {plan['threads']}>"
    if plan["passes"] == 5:
        z_ok = fast and pow2(pz) and 2 <= pz <= (64 if t == "float" else 32)
        if z_ok:
            # FP64 lines whose upper half is zero: two lanes per line
            if t == "double" and pz in (16, 32) and 2 * nz <= pz:
                return f"mm::k_kspace_z_split<{t}, {pz}>"
            return f"mm::k_kspace_z<{t}, {pz}>"
        if fast and pz in (128, 256, 512, 1024) and 2 * nz <= pz and not (t == "double" and pz == 1024):
            # long z lines: C columns a work-group, as many as the threads and LDS allow
            cols = {"float": {128: 32, 256: 16, 512: 4, 1024: 2}, "double": {128: 16, 256: 8, 512: 4}}[t][pz]
            return f"mm::k_kspace_zl<{t}, {pz}, {cols}>"
        if fast and pz in (128, 256, 512, 1024):
            return f"mm::k_kspace_fixed<{t}, {512 if pz == 512 else 256}, {pz}>"
        return f"mm::k_kspace<{t}, {plan['threads']}>"
    if plan.get("two_plane"):  # two cells thick: the two-plane y k-space pass
        return f"mm::k_kspace_y2<{t}, {py}, {b(2 * ny > py)}>"
    if pz > 1:  # three passes on a 3-D grid: the fused y-z pass
        return f"mm::k_kspace_yz<{t}, {plan['threads']}>"
    ky_ok = fast and pow2(py) and 16 <= py <= 1024
    return f"mm::k_kspace_y<{t}, {py}, {b(2 * ny > py)}>" if ky_ok else f"mm::k_kspace<{t}, {plan['threads']}>"


def kernel_key(name: str) -> str:
    """rocprofv3's demangled name without 'void ' and the argument list."""
    name = name[5:] if name.startswith("void ") else name
    if not name.endswith(")"):
        return name
    # the argument list is the last top-level parenthesis group
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        depth += name[i] == ")"
        depth -= name[i] == "("
        if depth == 0:
            return name[:i]
    return name


def summarize_rocprof(run_dir: str, out_dir: str, command: str) -> str:
    """Writes a summary of one profiled bench run: kernel-trace statistics
    (run_dir/kt), FETCH_SIZE (run_dir/pf) and WRITE_SIZE (run_dir/pw) per dispatch,
    both scaled by what they read for the 1 GiB device copy of the same run, and
    the bench line of the kernel-trace run (run_dir/kt.log)."""
    import csv
    import glob
    from collections import defaultdict

    def one(pattern):
        found = glob.glob(os.path.join(run_dir, pattern), recursive=True)
        if not found:
            raise SystemExit(f"no {pattern} under {run_dir}")
        return found[0]

    stats = list(csv.DictReader(open(one("kt/**/*kernel_stats.csv"))))
    line = [l for l in open(os.path.join(run_dir, "kt.log")) if l.startswith("{")][-1]
    b = json.loads(line)

    def counter(pattern, name):
        per = defaultdict(list)
        for r in csv.DictReader(open(one(pattern))):
            if r["Counter_Name"] == name:
                per[kernel_key(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return per

    fetch = counter("pf/**/*counter_collection.csv", "FETCH_SIZE")
    write = counter("pw/**/*counter_collection.csv", "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    scale = {"FETCH_SIZE": (1 << 30) / (max(fetch[copy]) * 1024),
             "WRITE_SIZE": (1 << 30) / (max(write[copy]) * 1024)}
    rl = b["roofline"]
    dom = rl["kernel"]
    workload = b["config"]["workload"]
    cells = grid_cells(b["plan"], workload)
    ab = {mm_kernel_symbol(k, b["dtype"], b["plan"], cells): v for k, v in b["algorithmic_bytes"].items()}
    rows, kernels = [], {}
    for k in sorted(set(fetch) & set(write) - {copy}):
        f = sum(fetch[k]) / len(fetch[k])
        w = sum(write[k]) / len(write[k])
        hbm = 1024 * (f * scale["FETCH_SIZE"] + w * scale["WRITE_SIZE"])
        tu = next((t for prefix, t in KERNEL_TU if k.startswith(prefix)), None)
        kernels[k] = {"dispatches": len(fetch[k]), "fetch_kib": f, "write_kib": w,
                      "hbm_bytes_per_launch": hbm,
                      "sources_sha256": b["sources_sha256"].get(tu) if tu else None}
        if k in ab:
            kernels[k]["algorithmic_bytes_per_launch"] = ab[k]
        st = [r for r in stats if kernel_key(r["Name"]) == k]
        if st:
            kernels[k]["avg_ns"] = float(st[0]["AverageNs"])
        rows.append((k, len(fetch[k]), f, w, hbm, ab.get(k)))
    short = dom.split("::")[-1].split("<")[0].replace("k_", "")
    tag = f"{short}_{b['config']['workload'].split(' cells')[0].replace(' ', '_')}_{b['dtype']}"
    path = os.path.join(out_dir, tag + ".md")
    lines = [f"# {dom} and the other kernels of one RK4 step: {workload}", "",
             "Commands:", "",
             "```", command.strip(), "```", "",
             "## Kernel time (`rocprofv3 --kernel-trace --stats`)", "",
             "| kernel | calls | avg µs | % of GPU time |", "|---|---|---|---|"]
    def short(name):
        return name if len(name) <= 90 else name[:87] + "..."

    for r in stats[:14]:
        lines.append(f"| `{short(kernel_key(r['Name']))}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} "
                     f"| {float(r['Percentage']):.1f} |")
    dom_rows = [r for r in stats if kernel_key(r["Name"]) == dom]
    if dom_rows:
        lines += ["", f"Dominant kernel `{dom}`: rocprofv3 average {float(dom_rows[0]['AverageNs']) / 1e3:.1f} µs"
                      f" over {dom_rows[0]['Calls']} launches; the bench's HIP events in the same run "
                      f"{1e3 * rl['avg_launch_ms']:.1f} µs over {rl['launches_timed']} launches."]
    lines += ["", "## HBM traffic per dispatch (`rocprofv3 --pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
              f"Calibration on the 1 GiB device copy of the same run: FETCH_SIZE reads "
              f"{max(fetch[copy]):.1f} KiB (scale {scale['FETCH_SIZE']:.4f}), WRITE_SIZE "
              f"{max(write[copy]):.1f} KiB (scale {scale['WRITE_SIZE']:.4f}). HBM bytes = 1024 · "
              f"(FETCH · scale + WRITE · scale).", "",
              "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM MB | algorithmic MB | HBM / algorithmic |",
              "|---|---|---|---|---|---|---|"]
    for k, n, f, w, hbm, a in sorted(rows, key=lambda r: -r[4]):
        ratio = f"{hbm / a:.3f}" if a else ""
        am = f"{a / 1e6:.1f}" if a else ""
        lines.append(f"| `{short(k)}` | {n} | {f:.0f} | {w:.0f} | {hbm / 1e6:.1f} | {am} | {ratio} |")
    lines += ["", f"Bench line of the kernel-trace run: value {b['value']:.4g} {b['unit']}, "
                  f"{b['ms_per_step']:.3f} ms per step (profiler attached).", "",
              "Record read by `bench.py` for `roofline.traffic` (a kernel's entry holds while "
              "its translation unit and headers hash to its `sources_sha256`):", "", "```json",
              json.dumps({"workload": workload, "precision": b["dtype"], "copy_scale": scale,
                          "kernels": kernels}, indent=1), "```", ""]
    os.makedirs(out_dir, exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines))
    return path


def summarize_batch_rocprof(run_dir: str, out_dir: str, command: str) -> str:
    """Summary of one profiled batched leg (bench.py --leg batched): per-kernel
    time (run_dir/kt), HBM bytes per dispatch from FETCH_SIZE (run_dir/pf) and
    WRITE_SIZE (run_dir/pw) with the counter scale of the 1 GiB device copy of
    the main summary (FETCH x2, WRITE x1), their sum over one RK4 step, and the
    share of the step's span the GPU sits between kernels."""
    import csv
    import glob
    from collections import defaultdict

    def one(pattern):
        found = glob.glob(os.path.join(run_dir, pattern), recursive=True)
        if not found:
            raise SystemExit(f"no {pattern} under {run_dir}")
        return found[0]

    stats = {kernel_key(r["Name"]): r for r in csv.DictReader(open(one("kt/**/*kernel_stats.csv")))}
    line = [l for l in open(os.path.join(run_dir, "kt.log")) if l.startswith("{")][-1]
    b = json.loads(line)

    def counter(pattern, name):
        per = defaultdict(list)
        for r in csv.DictReader(open(one(pattern))):
            if r["Counter_Name"] == name:
                per[kernel_key(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return per

    fetch = counter("pf/**/*counter_collection.csv", "FETCH_SIZE")
    write = counter("pw/**/*counter_collection.csv", "WRITE_SIZE")
    rows = []
    for k in sorted(set(fetch) & set(write) & set(stats)):
        if not k.startswith("mm::kb"):
            continue
        hbm = 1024 * (COPY_SCALE["FETCH_SIZE"] * sum(fetch[k]) / len(fetch[k]) +
                      COPY_SCALE["WRITE_SIZE"] * sum(write[k]) / len(write[k]))
        t = float(stats[k]["AverageNs"])
        rows.append((t, k, int(stats[k]["Calls"]), hbm))
    rows.sort(reverse=True)
    trace = [r for r in csv.DictReader(open(one("kt/**/*kernel_trace.csv"))) if r["Kernel_Name"].startswith(
        ("void mm::kb", "mm::kb"))]
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace)
    gaps = [int(y["Start_Timestamp"]) - int(x["End_Timestamp"]) for x, y in zip(trace, trace[1:])]
    idle = sum(g for g in gaps if 0 < g < 200000)   # longer gaps: host syncs between runs
    step_us = sum(4 * t for t, _, calls, _ in rows if calls) / 1e3
    step_mb = sum(4 * hbm for _, _, _, hbm in rows) / 1e6
    lines = [f"# Batched step: {b['grids']} grids, {b['cells']} cells, {b['padding']} padding, {b['passes']}", "",
             "Commands:", "", "```", command.strip(), "```", "",
             "## Kernels of one field evaluation and LLG stage (four per RK4 step)", "",
             "| kernel | calls | avg µs | HBM MB per launch | GB/s |", "|---|---|---|---|---|"]
    for t, k, calls, hbm in rows:
        lines.append(f"| `{k}` | {calls} | {t / 1e3:.1f} | {hbm / 1e6:.1f} | {hbm / t:.0f} |")
    lines += ["", f"Sum over one RK4 step (4 launches of each kernel): {step_us:.0f} µs of kernel time, "
                  f"{step_mb:.0f} MB of HBM traffic ({step_mb / step_us * 1e3:.0f} GB/s); "
                  f"the algorithmic model gives {b['step_model_bytes'] / 1e6:.0f} MB per step.",
              f"Between consecutive batched kernels the GPU is idle {100 * idle / (idle + busy):.2f}% of the "
              f"time (gaps under 200 µs, graph replay): the step is kernel time, not launch gaps.",
              "", f"Bench line of the kernel-trace run: {b['value']:.4g} {b['unit']}, {b['ms_per_step']:.3f} ms "
                  f"per step (profiler attached).", ""]
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"batched_{b['grids']}_grids_{b['padding'].split()[0]}_f32.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines))
    return path


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-batch-rocprof":
        # bench.py --summarize-batch-rocprof RUN_DIR OUT_DIR "COMMANDS"
        print(summarize_batch_rocprof(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif len(sys.argv) > 1 and sys.argv[1] == "--summarize-rocprof":
        # bench.py --summarize-rocprof RUN_DIR OUT_DIR "COMMANDS"
        print(summarize_rocprof(sys.argv[2], sys.argv[3], sys.argv[4]))
    else:
        main()
