"""Helpers shared by the GPU tests: error metrics and oracle problems."""
import numpy as np

import oracle


def rel_max(a, b):
    """max |a - b| / max |b|  (the field metric: relative to the largest entry)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def problem(nx, ny, nz, cell, Ms=8e5, A=1.3e-11, Ku=0.0, alpha=0.5, gamma=2.211e5,
            hext=(0.0, 0.0, 0.0), demag=True, ku_map=None):
    return oracle.Problem(nx, ny, nz, cell, Ms=Ms, A=A, Ku=Ku, alpha=alpha, gamma=gamma,
                          hext=tuple(hext), demag=demag, ku_map=ku_map)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
