"""Force-error and conservation metrics used to compare the GPU library with
the oracle (test infrastructure)."""
from __future__ import annotations

import numpy as np


def force_errors(got, ref, scale) -> dict:
    """got, ref: (3, k) accelerations of the same targets; scale: (k,) the
    oracle's A_i = sum_j |f_ij|.

    eps_rms  = sqrt(mean_i |a_i - a_i^ref|^2 / |a_i^ref|^2)
    eps_norm = ||a - a_ref||_2 / ||a_ref||_2
    eps_cond = max_i |a_i - a_i^ref| / A_i
    eps_max  = max_i |a_i - a_i^ref| / |a_i^ref|
    """
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.sqrt(((got - ref) ** 2).sum(0))
    r = np.sqrt((ref ** 2).sum(0))
    ok = r > 0
    A = np.asarray(scale, dtype=np.float64)
    return {
        "eps_rms": float(np.sqrt(np.mean((d[ok] / r[ok]) ** 2))) if ok.any() else 0.0,
        "eps_norm": float(np.linalg.norm(d) / np.linalg.norm(r)) if ok.any() else 0.0,
        "eps_cond": float(np.max(d[A > 0] / A[A > 0])) if (A > 0).any() else float(np.max(d, initial=0.0)),
        "eps_max": float(np.max(d[ok] / r[ok])) if ok.any() else 0.0,
    }
