"""Long integrations that follow the conserved quantities and the disk's
surface density over time: the measurements behind the paper's Table 2
(largest deviation of total momentum, angular momentum and energy over a
run), Figs. 5-6 (their time series and the centre of mass) and Fig. 7
(surface-density maps of single- against double-precision runs).

Everything on the device goes through the library: ``nbody_step_kdk`` for
the steps, ``nbody_diag`` for E, P, L and the centre of mass (float64 in
every precision mode) and ``nbody_surface_density`` for the maps.  The host
only collects the diagnostics and compares maps.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import nbody as nb


@dataclass
class Grid:
    """An nx-by-ny map over [x0, x0 + nx w) x [y0, y0 + ny w), cell width w."""
    nx: int = 256
    ny: int = 256
    x0: float = -6.0
    y0: float = -6.0
    w: float = 12.0 / 256

    def args(self):
        return (self.nx, self.ny, self.x0, self.y0, 1.0 / self.w, 1.0 / self.w)


@dataclass
class Record:
    steps: list = field(default_factory=list)
    E: list = field(default_factory=list)
    P: list = field(default_factory=list)      # (Px, Py, Pz)
    Lz: list = field(default_factory=list)
    com: list = field(default_factory=list)    # (x, y, z)
    maps: dict = field(default_factory=dict)   # step -> (ny, nx) uint32 counts
    busy_s: float = 0.0                        # wall time of the step calls only
    evals: int = 0
    final: dict | None = None                  # host copy of the last state
    done: int = 0                              # steps taken so far

    def add(self, step: int, d: dict) -> None:
        self.steps.append(step)
        self.E.append(d["E"])
        self.P.append((d["Px"], d["Py"], d["Pz"]))
        self.Lz.append(d["Lz"])
        self.com.append((d["Cx"], d["Cy"], d["Cz"]))

    def deviations(self) -> dict:
        """Per-sample deviations from the initial values: |P - P0|,
        |Lz - Lz0| / |Lz0|, |E - E0| / |E0| and |com - com0|."""
        P = np.asarray(self.P)
        C = np.asarray(self.com)
        E = np.asarray(self.E)
        L = np.asarray(self.Lz)
        return {
            "dP_abs": np.sqrt(((P - P[0]) ** 2).sum(1)),
            "dL_rel": np.abs(L - L[0]) / abs(L[0]),
            "dE_rel": np.abs(E - E[0]) / abs(E[0]),
            "dcom_abs": np.sqrt(((C - C[0]) ** 2).sum(1)),
        }

    def table2(self) -> dict:
        """Largest deviations over the run (the columns of Table 2)."""
        return {k + "_max": float(v.max()) for k, v in self.deviations().items()}

    def save(self, stem: str) -> None:
        """Write the record (``stem``.json) and its maps (``stem``_maps.npz);
        the particle state is saved separately (``checkpoint``)."""
        import json
        with open(stem + ".json", "w") as f:
            json.dump({"steps": self.steps, "E": self.E, "P": self.P, "Lz": self.Lz, "com": self.com,
                       "busy_s": self.busy_s, "evals": self.evals}, f)
        np.savez_compressed(stem + "_maps.npz", **{str(k): v for k, v in self.maps.items()})

    @classmethod
    def load(cls, stem: str) -> "Record":
        import json
        with open(stem + ".json") as f:
            d = json.load(f)
        rec = cls(steps=d["steps"], E=d["E"], P=[tuple(p) for p in d["P"]], Lz=d["Lz"],
                  com=[tuple(c) for c in d["com"]], busy_s=d["busy_s"], evals=d["evals"])
        with np.load(stem + "_maps.npz", allow_pickle=False) as z:
            rec.maps = {int(k): z[k] for k in z.files}
        return rec


def run(ctx, ic: dict, prm: "nb.Params", dt: float, steps: int, every: int = 50, maps_at=(),
        grid: Grid | None = None, plan: dict | None = None, progress=None, resume=None,
        stop_at: int | None = None, deadline: float | None = None) -> Record:
    """Integrate ``ic`` for ``steps`` leapfrog steps of ``dt``, sampling the
    diagnostics every ``every`` steps (and at 0) and a surface-density map at
    each step count in ``maps_at``.  ``plan`` pins the launch plan of the
    pair sum for this size (cleared afterwards).

    A run can be cut into pieces: ``stop_at`` ends it early at that step
    (``Record.done`` tells where), and ``resume=(record, step)`` continues
    from a record and a state saved at ``step`` (``ic`` then holds that
    state, accelerations included, as ``checkpoint`` writes it); the pieces
    take the same steps as one run, bit for bit.  ``deadline`` (a
    ``time.perf_counter()`` value) also ends the run early, at the first
    sample point reached after it."""
    grid = grid or Grid()
    s = nb.System.from_arrays(ic)
    n = s.n
    if plan is not None:
        nb.nbody_plan_set(ctx, prm.prec, n, plan)
    try:
        want_maps = sorted(set(int(k) for k in maps_at if 0 <= k <= steps))
        if resume is None:
            rec = Record()
            nb.nbody_accel(ctx, s, prm)
            rec.add(0, nb.diag_dict(nb.nbody_diag(ctx, s, prm)))
            if 0 in want_maps:
                rec.maps[0] = _map(ctx, s, grid)
            done = 0
        else:
            rec, done = resume
        end = steps if stop_at is None else min(steps, stop_at)
        stops = sorted(set(list(range(every, steps, every)) + [steps] + want_maps) - {0})
        for stop in stops:
            if stop <= done:
                continue
            if stop > end:
                break
            k = stop - done
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nb.nbody_step_kdk(ctx, s, prm, dt, k)
            torch.cuda.synchronize()
            rec.busy_s += time.perf_counter() - t0
            rec.evals += k
            done = stop
            if done % every == 0 or done == steps:
                rec.add(done, nb.diag_dict(nb.nbody_diag(ctx, s, prm)))
            if done in want_maps:
                rec.maps[done] = _map(ctx, s, grid)
            if progress is not None:
                progress(done, rec)
            if deadline is not None and time.perf_counter() >= deadline and done % every == 0:
                break
        rec.final = s.numpy()
        rec.done = done
        return rec
    finally:
        if plan is not None:
            nb.nbody_plan_set(ctx, prm.prec, n, None)


def _map(ctx, s, grid: Grid) -> np.ndarray:
    out = nb.nbody_surface_density(ctx, s, *grid.args())
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).copy()


def compare_maps(a: np.ndarray, b: np.ndarray) -> dict:
    """|sigma_a - sigma_b| of two count maps of equal-mass particles, as a
    fraction of the total (sum |d| / sum a; half of it is the fraction of the
    mass that sits in different cells) and of the peak (max |d| / max a)."""
    a = a.astype(np.int64)
    b = b.astype(np.int64)
    d = np.abs(a - b)
    tot = max(int(a.sum()), 1)
    return {"l1_frac": float(d.sum() / tot), "max_frac": float(d.max() / max(int(a.max()), 1))}


def nonaxisymmetry(counts: np.ndarray, grid: Grid, rmax: float = 4.0) -> float:
    """Mass-weighted amplitude of the m = 2 Fourier mode of the map inside
    rmax, |sum w e^{2 i phi}| / sum w: 0 for an axisymmetric disk, larger as
    a bar or two-armed spiral grows."""
    ny, nx = counts.shape
    xc = grid.x0 + (np.arange(nx) + 0.5) * grid.w
    yc = grid.y0 + (np.arange(ny) + 0.5) * grid.w
    X, Y = np.meshgrid(xc, yc)
    R = np.hypot(X, Y)
    w = counts.astype(np.float64) * (R < rmax)
    tot = w.sum()
    if tot == 0:
        return 0.0
    return float(abs((w * np.exp(2j * np.arctan2(Y, X))).sum()) / tot)


def interactions_per_s(n: int, rec: Record) -> float:
    return rec.evals * float(n) * float(n) / rec.busy_s if rec.busy_s > 0 else math.nan
