"""MI355X-native finite-difference micromagnetic LLG step (arXiv:1501.07293).

Thin ctypes binding of ``libmmag.so`` (the C ABI declared in include/mmag.h).
PyTorch supplies device memory (the workspace and array arguments) and the
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: without the built library every call raises.

Arrays are torch tensors of shape (3, nz, ny, nx) in the handle's precision
(float32 for "f32", float64 for "f64") on the GPU; host numpy arrays are
accepted by ``set_m`` and converted.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmag.so")

MM_F32, MM_F64 = 0, 1
MM_NO_DEMAG, MM_USE_GRAPH, MM_GENERIC_FFT, MM_AUTOTUNE, MM_POW2_PAD = 0x1, 0x2, 0x4, 0x8, 0x10
MM_NEWELL, MM_PER_GRID_MATERIAL = 0x20, 0x40
MM_PERIODIC_X, MM_PERIODIC_Y, MM_PERIODIC_Z = 0x80, 0x100, 0x200
MM_FUSED_YZ = 0x400
MM_ONE_WG = 0x800
MM_SPLIT_STAGE = 0x2000
MM_FAST_PAD = 0x1000
MM_RK4, MM_EULER = 0, 1
MM_NOALLOC_SCRATCH_BYTES = 96 << 20  # static adjoint scratch of mm_backward_noalloc
TERMS = {"exch": 0, "anis": 1, "demag": 2, "ext": 3, "eff": 4}
KERNELS = {"x_fwd": 0, "y_fwd": 1, "kspace": 2, "y_inv": 3, "x_inv": 4, "llg": 5}

EXPORTS = ["mm_workspace_query", "mm_create", "mm_destroy", "mm_set_stream", "mm_set_m", "mm_get_m",
           "mm_set_hext", "mm_set_alpha", "mm_set_ku_map", "mm_step", "mm_step_euler", "mm_run_schedule",
           "mm_get_field",
           "mm_get_energy", "mm_get_mean_m", "mm_get_max_torque", "mm_get_plan", "mm_get_kernel_spectrum",
           "mm_demag_tensor", "mm_demag_tensor_newell", "mm_batch_workspace_query", "mm_batch_create", "mm_batch_destroy",
           "mm_batch_set_stream", "mm_batch_set_m", "mm_batch_get_m", "mm_batch_step", "mm_batch_get_field",
           "mm_batch_cells", "mm_batch_get_info", "mm_batch_get_grid_plan", "mm_rollout", "mm_adjoint_workspace_query", "mm_backward", "mm_backward_noalloc", "mm_normalize_backward",
           "mm_profile_begin", "mm_profile_sample", "mm_profile_end", "mm_kernel_name", "mm_status_string",
           "mm_last_error"]


class MMError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {status_name(status)} ({status}): {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("cell", ctypes.c_double)]


class Material(ctypes.Structure):
    _fields_ = [("Ms", ctypes.c_double), ("A", ctypes.c_double), ("Ku", ctypes.c_double),
                ("alpha", ctypes.c_double), ("gamma", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("px", ctypes.c_int32), ("py", ctypes.c_int32),
                ("pz", ctypes.c_int32), ("flags", ctypes.c_uint32), ("threads", ctypes.c_int32),
                ("x_lines", ctypes.c_int32), ("images", ctypes.c_int32)]


class Segment(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("h0", ctypes.c_double * 3), ("h1", ctypes.c_double * 3),
                ("alpha", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("px", ctypes.c_int32), ("py", ctypes.c_int32), ("pz", ctypes.c_int32),
                ("hx", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("spectrum_elems", ctypes.c_int64), ("passes", ctypes.c_int32),
                ("kernel_imag_ratio", ctypes.c_double), ("generic_fft", ctypes.c_int32),
                ("tuned", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("tuned_demag_ms", ctypes.c_double), ("x_lines", ctypes.c_int32),
                ("x_lines_inv", ctypes.c_int32), ("two_plane", ctypes.c_int32),
                ("fused_stage", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("n", ctypes.c_int32), ("pow2_pad", ctypes.c_int32),
                ("size_classes", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("fast_pad", ctypes.c_int32),
                ("tuned_demag_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmmag.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1501_07293_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mm_workspace_query": [ctypes.POINTER(Grid), ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)],
        "mm_create": [ctypes.POINTER(Grid), ctypes.POINTER(Material), ctypes.POINTER(Options), vp,
                      ctypes.c_size_t, vp, ctypes.POINTER(vp)],
        "mm_destroy": [vp],
        "mm_set_stream": [vp, vp],
        "mm_set_m": [vp, vp, ctypes.c_int],
        "mm_get_m": [vp, vp, ctypes.c_int],
        "mm_set_hext": [vp, ctypes.POINTER(dbl)],
        "mm_set_alpha": [vp, dbl],
        "mm_set_ku_map": [vp, vp, ctypes.c_int],
        "mm_step": [vp, i64, dbl],
        "mm_step_euler": [vp, i64, dbl],
        "mm_run_schedule": [vp, ctypes.POINTER(Segment), i32, i32, dbl, i64, vp, i64, ctypes.POINTER(i64)],
        "mm_get_field": [vp, i32, vp, ctypes.c_int],
        "mm_get_energy": [vp, ctypes.POINTER(dbl)],
        "mm_get_mean_m": [vp, ctypes.POINTER(dbl)],
        "mm_get_max_torque": [vp, ctypes.POINTER(dbl)],
        "mm_get_plan": [vp, ctypes.POINTER(PlanInfo)],
        "mm_get_kernel_spectrum": [vp, vp, ctypes.c_int],
        "mm_demag_tensor": [i32, i32, i32, vp, vp],
        "mm_demag_tensor_newell": [i32, i32, i32, vp, vp],
        "mm_batch_workspace_query": [i32, ctypes.POINTER(Grid), ctypes.POINTER(Options),
                                     ctypes.POINTER(ctypes.c_size_t)],
        "mm_batch_create": [i32, ctypes.POINTER(Grid), ctypes.POINTER(Material), ctypes.POINTER(dbl),
                            ctypes.POINTER(Options), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
        "mm_batch_destroy": [vp],
        "mm_batch_set_stream": [vp, vp],
        "mm_batch_set_m": [vp, vp, ctypes.c_int],
        "mm_batch_get_m": [vp, vp, ctypes.c_int],
        "mm_batch_step": [vp, i64, dbl],
        "mm_batch_get_field": [vp, i32, vp, ctypes.c_int],
        "mm_batch_cells": [vp, ctypes.POINTER(i64)],
        "mm_batch_get_info": [vp, ctypes.POINTER(BatchInfo)],
        "mm_batch_get_grid_plan": [vp, ctypes.c_int32, ctypes.POINTER(PlanInfo)],
        "mm_rollout": [vp, i64, dbl, i64, vp],
        "mm_adjoint_workspace_query": [vp, i64, ctypes.POINTER(ctypes.c_size_t)],
        "mm_backward": [vp, i64, dbl, i64, vp, vp, vp, vp, vp, ctypes.c_size_t],
        "mm_backward_noalloc": [vp, i64, dbl, i64, vp, vp, vp, vp],
        "mm_normalize_backward": [vp, vp, vp, vp],
        "mm_profile_begin": [vp, i32],
        "mm_profile_sample": [vp, i32],
        "mm_profile_end": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.mm_kernel_name.argtypes = [i32]
    lib.mm_kernel_name.restype = ctypes.c_char_p
    lib.mm_status_string.argtypes = [ctypes.c_int]
    lib.mm_status_string.restype = ctypes.c_char_p
    lib.mm_last_error.argtypes = []
    lib.mm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_name(s: int) -> str:
    return load_library().mm_status_string(s).decode()


def _check(st: int, where: str):
    if st != 0:
        raise MMError(st, where, load_library().mm_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1501_07293_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Sim:
    """One grid + material on one GPU (handle around mm_create / mm_step)."""

    def __init__(self, nx: int, ny: int, nz: int, cell: float, Ms: float = 8.0e5,
                 A: float = 1.3e-11, Ku: float = 0.0, alpha: float = 0.5, gamma: float = 2.211e5,
                 precision: str = "f32", pad: Sequence[int] = (0, 0, 0), demag: bool = True,
                 graph: bool = False, threads: int = 0, generic_fft: bool = False,
                 autotune: bool = False, x_lines: int = 0, pow2_pad: bool = False, fast_pad: bool = False,
                 tensor: str = "point", periodic: Sequence[bool] = (False, False, False),
                 images: int = 0, fused_yz: bool = False, one_wg: bool = False, split_stage: bool = False,
                 device: str = "cuda:0"):
        """periodic: per axis x, y, z, no zero padding and a wrapped exchange
        stencil; images: images on each side beyond the nearest one in the
        periodic demag sum (MM_PERIODIC_X/Y/Z)."""
        torch = _torch()
        lib = load_library()
        self._torch = torch
        self.device = torch.device(device)
        self.nx, self.ny, self.nz, self.cell, self.Ms = nx, ny, nz, cell, Ms
        self.N = nx * ny * nz
        self.shape = (3, nz, ny, nx)
        self.precision = precision
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self._grid = Grid(nx, ny, nz, cell)
        self._mat = Material(Ms, A, Ku, alpha, gamma)
        flags = ((0 if demag else MM_NO_DEMAG) | (MM_USE_GRAPH if graph else 0)
                 | (MM_GENERIC_FFT if generic_fft else 0) | (MM_AUTOTUNE if autotune else 0)
                 | (MM_POW2_PAD if pow2_pad else 0) | (MM_FAST_PAD if fast_pad else 0)
                 | _tensor_flag(tensor) | (MM_PERIODIC_X if periodic[0] else 0) | (MM_PERIODIC_Y if periodic[1] else 0)
                 | (MM_PERIODIC_Z if periodic[2] else 0) | (MM_FUSED_YZ if fused_yz else 0)
                 | (MM_ONE_WG if one_wg else 0) | (MM_SPLIT_STAGE if split_stage else 0))
        self._opt = Options(MM_F32 if precision == "f32" else MM_F64, pad[0], pad[1], pad[2], flags,
                            threads, x_lines, images)
        nbytes = ctypes.c_size_t()
        _check(lib.mm_workspace_query(ctypes.byref(self._grid), ctypes.byref(self._opt),
                                      ctypes.byref(nbytes)), "mm_workspace_query")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            _check(lib.mm_create(ctypes.byref(self._grid), ctypes.byref(self._mat),
                                 ctypes.byref(self._opt), self.workspace.data_ptr(), nbytes.value,
                                 _stream_ptr(torch, self.device), ctypes.byref(h)), "mm_create")
        self._h = h
        self._lib = lib
        # the applied field and damping the handle holds (None after run_schedule,
        # which leaves those of its last step)
        self._hext_now = (0.0, 0.0, 0.0)
        self._alpha_now = float(alpha)

    # ---------------------------------------------------------------- state
    def _sync_stream(self):
        _check(self._lib.mm_set_stream(self._h, _stream_ptr(self._torch, self.device)), "mm_set_stream")

    def set_m(self, m):
        torch = self._torch
        if isinstance(m, np.ndarray):
            m = torch.from_numpy(np.ascontiguousarray(m))
        t = m.to(device=self.device, dtype=self.dtype).contiguous().reshape(self.shape)
        self._sync_stream()
        _check(self._lib.mm_set_m(self._h, t.data_ptr(), 1), "mm_set_m")

    def get_m(self):
        out = self._torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_get_m(self._h, out.data_ptr(), 1), "mm_get_m")
        return out

    def set_hext(self, h: Sequence[float]):
        arr = (ctypes.c_double * 3)(*[float(v) for v in h])
        _check(self._lib.mm_set_hext(self._h, arr), "mm_set_hext")
        self._hext_now = tuple(arr[:])

    def set_alpha(self, alpha: float):
        _check(self._lib.mm_set_alpha(self._h, float(alpha)), "mm_set_alpha")
        self._alpha_now = float(alpha)

    def set_ku_map(self, ku):
        if ku is None:
            _check(self._lib.mm_set_ku_map(self._h, None, 0), "mm_set_ku_map")
            return
        torch = self._torch
        if isinstance(ku, np.ndarray):
            ku = torch.from_numpy(np.ascontiguousarray(ku))
        t = ku.to(device=self.device, dtype=self.dtype).contiguous().reshape(self.nz, self.ny, self.nx)
        self._sync_stream()
        _check(self._lib.mm_set_ku_map(self._h, t.data_ptr(), 1), "mm_set_ku_map")

    def step(self, nsteps: int, dt: float):
        self._sync_stream()
        _check(self._lib.mm_step(self._h, int(nsteps), float(dt)), "mm_step")

    def step_euler(self, nsteps: int, dt: float):
        """The paper's explicit Euler + renormalisation, nsteps steps."""
        self._sync_stream()
        _check(self._lib.mm_step_euler(self._h, int(nsteps), float(dt)), "mm_step_euler")

    def run_schedule(self, pieces, dt: float, every: int, method: str = "rk4"):
        """Runs the pieces of a time-dependent protocol; each piece is
        (steps, h0, h1, alpha) with the applied field ramping linearly from h0
        (A/m) at the piece's first step towards h1 (h1 = h0: constant).  Returns
        the trace, a float64 tensor (rows, 4) of {t [s], <m_x>, <m_y>, <m_z>}
        sampled after every `every`-th step."""
        torch = self._torch
        segs = (Segment * max(1, len(pieces)))()
        total = 0
        for q, (steps, h0, h1, alpha) in enumerate(pieces):
            segs[q].steps = int(steps)
            for c in range(3):
                segs[q].h0[c] = float(h0[c])
                segs[q].h1[c] = float(h1[c])
            segs[q].alpha = float(alpha)
            total += int(steps)
        cap = max(1, total // max(1, int(every)))
        trace = torch.empty((cap, 4), dtype=torch.float64, device=self.device)
        rows = ctypes.c_int64()
        self._sync_stream()
        self._hext_now = self._alpha_now = None
        _check(self._lib.mm_run_schedule(self._h, segs, len(pieces),
                                         MM_EULER if method == "euler" else MM_RK4, float(dt),
                                         int(every), trace.data_ptr(), cap, ctypes.byref(rows)),
               "mm_run_schedule")
        return trace[:rows.value]

    # --------------------------------------------------------------- readout
    def field(self, term: str = "eff"):
        out = self._torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_get_field(self._h, TERMS[term], out.data_ptr(), 1), "mm_get_field")
        return out

    def energy(self) -> np.ndarray:
        out = (ctypes.c_double * 5)()
        self._sync_stream()
        _check(self._lib.mm_get_energy(self._h, out), "mm_get_energy")
        return np.array(out[:])

    def mean_m(self) -> np.ndarray:
        out = (ctypes.c_double * 3)()
        self._sync_stream()
        _check(self._lib.mm_get_mean_m(self._h, out), "mm_get_mean_m")
        return np.array(out[:])

    def max_torque(self) -> float:
        """max over cells of |m x H_eff|, A/m (FP64 reduction on the GPU)."""
        out = ctypes.c_double()
        self._sync_stream()
        _check(self._lib.mm_get_max_torque(self._h, ctypes.byref(out)), "mm_get_max_torque")
        return out.value

    def plan(self) -> dict:
        p = PlanInfo()
        _check(self._lib.mm_get_plan(self._h, ctypes.byref(p)), "mm_get_plan")
        return {k: getattr(p, k) for k, _ in PlanInfo._fields_}

    def kernel_spectrum(self):
        p = self.plan()
        out = self._torch.empty(int(p["spectrum_elems"]), dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_get_kernel_spectrum(self._h, out.data_ptr(), 1), "mm_get_kernel_spectrum")
        if p["two_plane"]:
            return out.reshape(10, p["hx"], p["py"] // 2 + 1)
        return out.reshape(p["ncomp"], p["pz"] // 2 + 1, p["hx"], p["py"] // 2 + 1)

    # ----------------------------------------------------------- adjoint
    def rollout_ckpt(self, nsteps: int, dt: float, ckpt_every: int):
        """nsteps RK4 steps from the current m; returns the segment checkpoints."""
        nseg = (nsteps + ckpt_every - 1) // ckpt_every
        ck = self._torch.empty((nseg,) + self.shape, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_rollout(self._h, int(nsteps), float(dt), int(ckpt_every), ck.data_ptr()),
               "mm_rollout")
        return ck

    def backward(self, nsteps: int, dt: float, ckpt_every: int, ckpt, lam_final,
                 want_dm0: bool = True, noalloc: bool = False):
        """Reverse sweep: returns (dLoss/dKu per cell (float64, (nz, ny, nx)),
        dLoss/dm0 or None) for dLoss/dm_final = lam_final.  noalloc: call
        mm_backward_noalloc (the library's static scratch instead of a workspace
        allocated here)."""
        torch = self._torch
        lam = lam_final.to(device=self.device, dtype=self.dtype).contiguous()
        dku = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        dm0 = torch.empty(self.shape, dtype=self.dtype, device=self.device) if want_dm0 else None
        dm0_ptr = dm0.data_ptr() if dm0 is not None else None
        if noalloc:
            self._sync_stream()
            _check(self._lib.mm_backward_noalloc(self._h, int(nsteps), float(dt), int(ckpt_every),
                                                 ckpt.data_ptr(), lam.data_ptr(), dku.data_ptr(), dm0_ptr),
                   "mm_backward_noalloc")
            return dku, dm0
        nbytes = ctypes.c_size_t()
        _check(self._lib.mm_adjoint_workspace_query(self._h, int(ckpt_every), ctypes.byref(nbytes)),
               "mm_adjoint_workspace_query")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_backward(self._h, int(nsteps), float(dt), int(ckpt_every), ckpt.data_ptr(),
                                     lam.data_ptr(), dku.data_ptr(), dm0_ptr, ws.data_ptr(),
                                     nbytes.value), "mm_backward")
        return dku, dm0

    def normalize_backward(self, v, g_u):
        """dLoss/dv for u = v / |v| per cell (the normalisation set_m applies),
        given dLoss/du; both (3, nz, ny, nx) in the handle's precision."""
        torch = self._torch
        vv = v.to(device=self.device, dtype=self.dtype).contiguous()
        gu = g_u.to(device=self.device, dtype=self.dtype).contiguous()
        out = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_normalize_backward(self._h, vv.data_ptr(), gu.data_ptr(), out.data_ptr()),
               "mm_normalize_backward")
        return out

    # ------------------------------------------------------------- profiling
    def profile_begin(self, kernel: str, every: int = 1):
        """Time launches of `kernel` (one in `every`) until profile_end."""
        self._sync_stream()
        _check(self._lib.mm_profile_sample(self._h, int(every)), "mm_profile_sample")
        _check(self._lib.mm_profile_begin(self._h, KERNELS[kernel]), "mm_profile_begin")

    def profile_end(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.mm_profile_end(self._h, ctypes.byref(ms), ctypes.byref(n)), "mm_profile_end")
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSim:
    """Many independent grids of uneven sizes advanced together: one kernel launch
    per pass over all grids (handle around mm_batch_*).  Ms, A, Ku, alpha and gamma
    are each a number (every grid) or a sequence with one value per grid."""

    def __init__(self, grids: Sequence[Sequence[int]], cell: float, Ms: float = 8.0e5,
                 A: float = 1.3e-11, Ku: float = 0.0, alpha: float = 0.5, gamma: float = 2.211e5,
                 hext=None, precision: str = "f32", demag: bool = True, graph: bool = False,
                 pow2_pad: bool = False, fast_pad: bool = False, tensor: str = "point",
                 autotune: bool = False,
                 device: str = "cuda:0"):
        torch = _torch()
        lib = load_library()
        self._torch, self._lib = torch, lib
        self.device = torch.device(device)
        self.n = len(grids)
        self.shapes = [(3, int(g[2]), int(g[1]), int(g[0])) for g in grids]
        self.sizes = [3 * g[0] * g[1] * g[2] for g in grids]
        self.precision = precision
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        garr = (Grid * self.n)(*[Grid(int(g[0]), int(g[1]), int(g[2]), cell) for g in grids])
        self._grids = garr
        props = [Ms, A, Ku, alpha, gamma]
        per_grid = any(np.ndim(v) > 0 for v in props)
        if per_grid:
            cols = [np.broadcast_to(np.asarray(v, dtype=np.float64), (self.n,)) for v in props]
            self._mat = (Material * self.n)(*[Material(*(float(c[i]) for c in cols))
                                              for i in range(self.n)])
        else:
            self._mat = (Material * 1)(Material(*(float(v) for v in props)))
        flags = ((0 if demag else MM_NO_DEMAG) | (MM_USE_GRAPH if graph else 0)
                 | (MM_POW2_PAD if pow2_pad else 0) | (MM_FAST_PAD if fast_pad else 0)
                 | _tensor_flag(tensor) | (MM_PER_GRID_MATERIAL if per_grid else 0) | (MM_AUTOTUNE if autotune else 0))
        self._opt = Options(MM_F32 if precision == "f32" else MM_F64, 0, 0, 0, flags, 0, 0)
        h = np.zeros((self.n, 3)) if hext is None else np.ascontiguousarray(hext, dtype=np.float64)
        self._hext = (ctypes.c_double * (3 * self.n))(*h.reshape(-1).tolist())
        nbytes = ctypes.c_size_t()
        _check(lib.mm_batch_workspace_query(self.n, garr, ctypes.byref(self._opt), ctypes.byref(nbytes)),
               "mm_batch_workspace_query")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            hdl = ctypes.c_void_p()
            _check(lib.mm_batch_create(self.n, garr, self._mat, self._hext,
                                       ctypes.byref(self._opt), self.workspace.data_ptr(), nbytes.value,
                                       _stream_ptr(torch, self.device), ctypes.byref(hdl)),
                   "mm_batch_create")
        self._h = hdl
        c = ctypes.c_int64()
        _check(lib.mm_batch_cells(self._h, ctypes.byref(c)), "mm_batch_cells")
        self.cells = c.value

    def _sync_stream(self):
        _check(self._lib.mm_batch_set_stream(self._h, _stream_ptr(self._torch, self.device)),
               "mm_batch_set_stream")

    def info(self) -> dict:
        """The layout in use: padding family, pass family, autotune record."""
        p = BatchInfo()
        _check(self._lib.mm_batch_get_info(self._h, ctypes.byref(p)), "mm_batch_get_info")
        return {k: getattr(p, k) for k, _ in BatchInfo._fields_}

    def grid_plan(self, i: int) -> dict:
        """Padded sizes and schedule of grid i as the batch runs it."""
        p = PlanInfo()
        _check(self._lib.mm_batch_get_grid_plan(self._h, int(i), ctypes.byref(p)), "mm_batch_get_grid_plan")
        return {k: getattr(p, k) for k, _ in PlanInfo._fields_}

    def set_m(self, ms):
        """ms: list of per-grid (3, nz, ny, nx) arrays (or one flat array)."""
        torch = self._torch
        if isinstance(ms, (list, tuple)):
            flat = np.concatenate([np.asarray(m, dtype=np.float64).reshape(-1) for m in ms])
            t = torch.from_numpy(flat)
        else:
            t = ms if isinstance(ms, torch.Tensor) else torch.from_numpy(np.asarray(ms))
        t = t.to(device=self.device, dtype=self.dtype).contiguous().reshape(-1)
        assert t.numel() == sum(self.sizes)
        self._sync_stream()
        _check(self._lib.mm_batch_set_m(self._h, t.data_ptr(), 1), "mm_batch_set_m")

    def get_m_flat(self):
        out = self._torch.empty(sum(self.sizes), dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_batch_get_m(self._h, out.data_ptr(), 1), "mm_batch_get_m")
        return out

    def get_m(self):
        flat = self.get_m_flat()
        out, off = [], 0
        for shp, sz in zip(self.shapes, self.sizes):
            out.append(flat[off:off + sz].reshape(shp))
            off += sz
        return out

    def step(self, nsteps: int, dt: float):
        self._sync_stream()
        _check(self._lib.mm_batch_step(self._h, int(nsteps), float(dt)), "mm_batch_step")

    def field(self, term: str = "eff"):
        """One effective-field term of every grid, A/m: list of (3, nz, ny, nx)."""
        flat = self._torch.empty(sum(self.sizes), dtype=self.dtype, device=self.device)
        self._sync_stream()
        _check(self._lib.mm_batch_get_field(self._h, TERMS[term], flat.data_ptr(), 1),
               "mm_batch_get_field")
        out, off = [], 0
        for shp, sz in zip(self.shapes, self.sizes):
            out.append(flat[off:off + sz].reshape(shp))
            off += sz
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def demag_tensor(nx: int, ny: int, nz: int, device: str = "cuda:0", tensor: str = "point"):
    """Demag tensor on the GPU in FP64: (6, 2nz-1, 2ny-1, 2nx-1); tensor "point" is
    Eqs. 10-11, "newell" the cell-averaged tensor."""
    torch = _torch()
    lib = load_library()
    out = torch.empty((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1), dtype=torch.float64, device=device)
    fn = lib.mm_demag_tensor_newell if _tensor_flag(tensor) else lib.mm_demag_tensor
    _check(fn(nx, ny, nz, out.data_ptr(), _stream_ptr(torch, torch.device(device))), "mm_demag_tensor")
    return out


def _tensor_flag(tensor: str) -> int:
    if tensor not in ("point", "newell"):
        raise ValueError(f"tensor must be 'point' or 'newell', not {tensor!r}")
    return MM_NEWELL if tensor == "newell" else 0


def kernel_name(k: int) -> str:
    return load_library().mm_kernel_name(k).decode()


def _rollout_function():
    import torch

    class Rollout(torch.autograd.Function):
        """m_final = RK4^nsteps(m0 / |m0|; Ku map) on the GPU, with the hand-written
        adjoint (checkpoint every ckpt_every steps, segments recomputed in the
        backward pass).  Gradients flow to the Ku map (J/m^3, per cell) and to m0
        as given (through the per-cell normalisation the forward applies).  The
        Ku map, applied field and damping of the forward are kept and restored on
        the handle before the reverse sweep, so other rollouts or parameter
        changes on the same handle between forward and backward do not alter
        the gradient; the handle keeps them afterwards."""

        @staticmethod
        def forward(ctx, ku, m0, sim, nsteps, dt, ckpt_every):
            if sim._hext_now is None or sim._alpha_now is None:
                raise RuntimeError("rollout: set the applied field and damping (set_hext, set_alpha) "
                                   "after run_schedule")
            ku_used = ku.detach().to(device=sim.device, dtype=sim.dtype).contiguous().clone()
            m0_used = m0.detach().to(device=sim.device, dtype=sim.dtype).contiguous().clone()
            sim.set_ku_map(ku_used)
            sim.set_m(m0_used)
            ck = sim.rollout_ckpt(nsteps, dt, ckpt_every)
            ctx.sim, ctx.nsteps, ctx.dt, ctx.ckpt_every = sim, nsteps, dt, ckpt_every
            ctx.hext, ctx.alpha = sim._hext_now, sim._alpha_now
            ctx.save_for_backward(ck, ku_used, m0_used)
            ctx.ku_dtype, ctx.m0_dtype = ku.dtype, m0.dtype
            return sim.get_m()

        @staticmethod
        def backward(ctx, grad_m):
            ck, ku_used, m0_used = ctx.saved_tensors
            sim = ctx.sim
            sim.set_ku_map(ku_used)
            sim.set_hext(ctx.hext)
            sim.set_alpha(ctx.alpha)
            dku, dm0 = sim.backward(ctx.nsteps, ctx.dt, ctx.ckpt_every, ck, grad_m,
                                    want_dm0=ctx.needs_input_grad[1])
            gku = dku.to(ctx.ku_dtype) if ctx.needs_input_grad[0] else None
            gm0 = sim.normalize_backward(m0_used, dm0).to(ctx.m0_dtype) if dm0 is not None else None
            return gku, gm0, None, None, None, None

    return Rollout


_ROLLOUT = None


def rollout(sim: Sim, ku, m0, nsteps: int, dt: float, ckpt_every: int = 50):
    """Differentiable RK4 rollout (torch.autograd): returns m after nsteps."""
    global _ROLLOUT
    if _ROLLOUT is None:
        _ROLLOUT = _rollout_function()
    return _ROLLOUT.apply(ku, m0, sim, nsteps, dt, ckpt_every)
