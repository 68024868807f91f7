"""Checkpoint and resume of a particle state.

A snapshot holds everything the next step reads: positions, velocities,
masses and the current accelerations (the leapfrog reuses a(t) from the
previous step instead of recomputing it), the jerks when the system carries
them (the Hermite scheme reuses a and j of the last predicted state), plus the
time, the step count and the parameters.  Resuming from a snapshot therefore continues bit for bit
like an uninterrupted run.  Files are plain ``.npz`` archives (no pickles).

A compact snapshot (``compact=True``) keeps only positions and velocities, and
the masses as one number when they are all equal: 48 B per particle instead
of 80.  Loading it recomputes the accelerations with ``nbody_accel`` under the
plan the context holds for the system; the pair sums are deterministic, so for
a leapfrog run (whose stored a is the sum at the stored positions) this gives
the same bits as the full snapshot.
"""
from __future__ import annotations

import json

import numpy as np

from . import nbody as nb

_ARRAYS = ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az")
_JERK = ("jx", "jy", "jz")


def save(path: str, sys: "nb.System", prm: "nb.Params", t: float = 0.0, step: int = 0,
         compact: bool = False, **meta) -> None:
    """Write the state of ``sys`` (synchronises with the device); ``compact``
    leaves out the accelerations (and the jerks), and the masses when they are
    all equal."""
    info = {"t": float(t), "step": int(step), "params": prm.__dict__, "meta": meta}
    if compact:
        arrs = {k: sys.t[k].cpu().numpy() for k in _ARRAYS[:6]}
        m = sys.t["m"].cpu().numpy()
        if m.size and np.all(m == m[0]):
            info["m_equal"] = float(m[0])
            info["n"] = int(m.size)
        else:
            arrs["m"] = m
        info["compact"] = True
    else:
        arrs = {k: sys.t[k].cpu().numpy() for k in _ARRAYS}
        if all(sys.t.get(k) is not None for k in _JERK):
            arrs.update({k: sys.t[k].cpu().numpy() for k in _JERK})
    np.savez(path, info=np.array(json.dumps(info)), **arrs)


def load(path: str, device="cuda", ctx=None):
    """Return (System, Params, t, step, meta) from a snapshot.  A compact
    snapshot needs ``ctx``: its accelerations are recomputed there."""
    with np.load(path, allow_pickle=False) as z:
        info = json.loads(str(z["info"]))
        arrs = {k: z[k] for k in _ARRAYS + _JERK if k in z.files}
    prm = nb.Params(**info["params"])
    if info.get("compact"):
        if ctx is None:
            raise ValueError(f"{path} is a compact snapshot: pass ctx to recompute its accelerations")
        if "m" not in arrs:
            arrs["m"] = np.full(info["n"], info["m_equal"])
        for k in ("ax", "ay", "az"):
            arrs[k] = np.zeros_like(arrs["x"])
    sys = nb.System.from_arrays(arrs, device=device)
    if info.get("compact"):
        nb.nbody_accel(ctx, sys, prm)
    return sys, prm, info["t"], info["step"], info["meta"]
