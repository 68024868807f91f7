"""Checkpoint and resume of a particle state.

A snapshot holds everything the next step reads: positions, velocities,
masses and the current accelerations (the leapfrog reuses a(t) from the
previous step instead of recomputing it), the jerks when the system carries
them (the Hermite scheme reuses a and j of the last predicted state), plus the
time, the step count and the parameters.  Resuming from a snapshot therefore continues bit for bit
like an uninterrupted run.  Files are plain ``.npz`` archives (no pickles).
"""
from __future__ import annotations

import json

import numpy as np

from . import nbody as nb

_ARRAYS = ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az")
_JERK = ("jx", "jy", "jz")


def save(path: str, sys: "nb.System", prm: "nb.Params", t: float = 0.0, step: int = 0, **meta) -> None:
    """Write the state of ``sys`` (synchronises with the device)."""
    arrs = {k: sys.t[k].cpu().numpy() for k in _ARRAYS}
    if all(sys.t.get(k) is not None for k in _JERK):
        arrs.update({k: sys.t[k].cpu().numpy() for k in _JERK})
    info = {"t": float(t), "step": int(step), "params": prm.__dict__, "meta": meta}
    np.savez(path, info=np.array(json.dumps(info)), **arrs)


def load(path: str, device="cuda"):
    """Return (System, Params, t, step, meta) from a snapshot."""
    with np.load(path, allow_pickle=False) as z:
        info = json.loads(str(z["info"]))
        arrs = {k: z[k] for k in _ARRAYS + _JERK if k in z.files}
    sys = nb.System.from_arrays(arrs, device=device)
    prm = nb.Params(**info["params"])
    return sys, prm, info["t"], info["step"], info["meta"]
