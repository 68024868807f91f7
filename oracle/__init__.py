"""CPU FP64 oracle for the direct-sum N-body step -- TEST INFRASTRUCTURE.

This package is the checker, not the product: only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It wraps
``nbody_oracle.c`` (plain C, scalar FP64, IEEE sqrt/div, no FMA contraction)
through ctypes and shares no code with the GPU library.

Functions follow the paper (Khrapov, Khoperskov & Khoperskov 2018):
``accel`` -- Eqs. (1)-(2); ``step_kdk`` -- Eqs. (5)-(7); ``step_o4`` -- the
fourth-order scheme named in the abstract (triple-jump composition);
``accel_jerk``, ``State.step_hermite``, ``State.step_rk4`` -- the other
readings of that scheme (fourth-order Hermite on the jerk, classical RK4);
``diag`` -- Eqs. (8)-(10) plus centre of mass; ``surface_density`` -- the
maps of Section 3 (Fig. 7); ``halo_accel`` -- the optional fixed external
field of the disk workloads (not in the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Portable x86-64 level so the library built here also runs on other hosts.
CFLAGS = ["-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]

YOSHIDA_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
YOSHIDA_W0 = 1.0 - 2.0 * YOSHIDA_W1


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (seconds)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Halo(ctypes.Structure):
    _fields_ = [("on", ctypes.c_int), ("v2", ctypes.c_double), ("rc", ctypes.c_double)]


@dataclass
class Halo:
    v2: float
    rc: float


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int64)
_i64, _dbl, _int, _int32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int32


def load_library(path: str | None = None):
    """(Re)load the oracle library; ``path`` selects another build of the
    same source (the mutation tests use this to load planted mistakes)."""
    global _lib
    _lib = None
    return _load(path)


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        path = path or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(path)
        lib.orc_accel.argtypes = [_i64, _D, _D, _D, _D, _dbl, _dbl, _I, _i64, _int, _D, _D, _D, _D,
                                  _D, _int]
        lib.orc_halo_accel.argtypes = [_i64, _D, _D, _D, _dbl, _dbl, _D, _D, _D, _D]
        hp = ctypes.POINTER(_Halo)
        lib.orc_step_kdk.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _dbl, _dbl, hp,
                                     _dbl, _i64, _int, _int, _int]
        lib.orc_step_o4.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _dbl, _dbl, hp,
                                    _dbl, _i64, _dbl, _dbl, _int, _int]
        lib.orc_diag.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _dbl, _dbl, hp, _D, _int]
        lib.orc_accel_jerk.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _dbl, _dbl, hp, _I, _i64, _D, _D,
                                       _D, _D, _D, _D, _D, _D, _int]
        lib.orc_step_hermite.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _dbl,
                                         _dbl, hp, _dbl, _i64, _int]
        lib.orc_step_rk4.argtypes = [_i64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _dbl, _dbl, hp, _dbl,
                                     _i64, _int]
        lib.orc_surface_density.argtypes = [_i64, _D, _D, _int32, _int32, _dbl, _dbl, _dbl, _dbl,
                                            ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_force_evals.restype = _i64
        lib.orc_max_threads.restype = _int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _halo(h: Halo | None):
    s = _Halo(0, 0.0, 0.0) if h is None else _Halo(1, float(h.v2), float(h.rc))
    return ctypes.byref(s), s


def max_threads() -> int:
    return _load().orc_max_threads()


def accel(x, y, z, m, G=1.0, eps=0.0, rows=None, reverse_j=False, want_phi=False,
          want_scale=False, nthreads=0):
    """Eqs. (1)-(2). Returns (ax, ay, az[, phi][, A]) for all i or for ``rows``."""
    lib = _load()
    x, y, z, m = map(_f64, (x, y, z, m))
    n = x.size
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cnt = rows.size
        rp = rows.ctypes.data_as(_I)
    else:
        cnt = n
        rp = None
    ax, ay, az = np.zeros(cnt), np.zeros(cnt), np.zeros(cnt)
    phi = np.zeros(cnt) if want_phi else None
    A = np.zeros(cnt) if want_scale else None
    lib.orc_accel(n, _p(x), _p(y), _p(z), _p(m), G, eps, rp, cnt, int(reverse_j), _p(ax), _p(ay),
                  _p(az), _p(phi) if phi is not None else None, _p(A) if A is not None else None,
                  nthreads)
    out = [ax, ay, az]
    if want_phi:
        out.append(phi)
    if want_scale:
        out.append(A)
    return tuple(out)


def halo_accel(x, y, z, halo: Halo, want_phi=False):
    lib = _load()
    x, y, z = map(_f64, (x, y, z))
    n = x.size
    ax, ay, az = np.zeros(n), np.zeros(n), np.zeros(n)
    phi = np.zeros(n) if want_phi else None
    lib.orc_halo_accel(n, _p(x), _p(y), _p(z), halo.v2, halo.rc, _p(ax), _p(ay), _p(az),
                       _p(phi) if phi is not None else None)
    return (ax, ay, az, phi) if want_phi else (ax, ay, az)


def total_accel(s: dict, G=1.0, eps=0.0, halo: Halo | None = None, reverse_j=False, nthreads=0):
    ax, ay, az = accel(s["x"], s["y"], s["z"], s["m"], G, eps, reverse_j=reverse_j,
                       nthreads=nthreads)
    if halo is not None:
        hx, hy, hz = halo_accel(s["x"], s["y"], s["z"], halo)
        ax, ay, az = ax + hx, ay + hy, az + hz
    return ax, ay, az


class State:
    """Particle state as FP64 numpy arrays (x, y, z, vx, vy, vz, m, ax, ay, az)."""

    KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az")

    def __init__(self, ic: dict, G=1.0, eps=0.0, halo: Halo | None = None, nthreads=0,
                 reverse_j=False):
        self.a = {k: _f64(ic[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
        self.n = self.a["x"].size
        self.G, self.eps, self.halo = float(G), float(eps), halo
        self.nthreads, self.reverse_j = nthreads, reverse_j
        ax, ay, az = total_accel(self.a, G, eps, halo, reverse_j, nthreads)
        self.a["ax"], self.a["ay"], self.a["az"] = ax, ay, az

    def __getitem__(self, k):
        return self.a[k]

    def _ptrs(self):
        a = self.a
        return [_p(a[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az")]

    def step_kdk(self, dt, nsteps=1, paper_form=False):
        hp, _keep = _halo(self.halo)
        _load().orc_step_kdk(self.n, *self._ptrs(), self.G, self.eps, hp, dt, nsteps,
                             int(paper_form), int(self.reverse_j), self.nthreads)
        return self

    def init_jerk(self):
        """Acceleration and jerk at the current state (for step_hermite)."""
        a = self.a
        out = accel_jerk(a, self.G, self.eps, self.halo, self.nthreads)
        for k, v in zip(("ax", "ay", "az", "jx", "jy", "jz"), out):
            a[k] = v
        return self

    def step_hermite(self, dt, nsteps=1):
        if "jx" not in self.a:
            self.init_jerk()
        hp, _keep = _halo(self.halo)
        a = self.a
        _load().orc_step_hermite(self.n, *self._ptrs(), _p(a["jx"]), _p(a["jy"]), _p(a["jz"]), self.G,
                                 self.eps, hp, dt, nsteps, self.nthreads)
        return self

    def step_rk4(self, dt, nsteps=1):
        hp, _keep = _halo(self.halo)
        _load().orc_step_rk4(self.n, *self._ptrs(), self.G, self.eps, hp, dt, nsteps, self.nthreads)
        return self

    def step_o4(self, dt, nsteps=1, w1=YOSHIDA_W1, w0=YOSHIDA_W0):
        hp, _keep = _halo(self.halo)
        _load().orc_step_o4(self.n, *self._ptrs(), self.G, self.eps, hp, dt, nsteps, w1, w0,
                            int(self.reverse_j), self.nthreads)
        return self

    def diag(self):
        return diag(self.a, self.G, self.eps, self.halo, self.nthreads)

    def copy(self):
        c = State.__new__(State)
        c.a = {k: v.copy() for k, v in self.a.items()}
        c.n, c.G, c.eps, c.halo = self.n, self.G, self.eps, self.halo
        c.nthreads, c.reverse_j = self.nthreads, self.reverse_j
        return c


DIAG_KEYS = ("K", "W", "Wext", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "Cx", "Cy", "Cz", "M")


def diag(s: dict, G=1.0, eps=0.0, halo: Halo | None = None, nthreads=0) -> dict:
    """Eqs. (8)-(10) and the centre of mass (see nbody_oracle.c)."""
    lib = _load()
    a = {k: _f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    out = np.zeros(14)
    hp, _keep = _halo(halo)
    lib.orc_diag(a["x"].size, _p(a["x"]), _p(a["y"]), _p(a["z"]), _p(a["vx"]), _p(a["vy"]),
                 _p(a["vz"]), _p(a["m"]), G, eps, hp, _p(out), nthreads)
    return dict(zip(DIAG_KEYS, out.tolist()))


def accel_jerk(s: dict, G=1.0, eps=0.0, halo: Halo | None = None, nthreads=0, want_scale=False, rows=None):
    """Acceleration (Eqs. (1)-(2)) and its time derivative along the motion,
    plus the halo's when given, for all particles or for ``rows``.  Returns
    (ax, ay, az, jx, jy, jz), and with want_scale also the sums of the
    self-gravity terms' magnitudes (A, J)."""
    lib = _load()
    a = {k: _f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    n = a["x"].size
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if r is None else r.size
    out = [np.zeros(cnt) for _ in range(8 if want_scale else 6)]
    hp, _keep = _halo(halo)
    sc = [_p(o) for o in out[6:]] if want_scale else [None, None]
    rp = None if r is None else r.ctypes.data_as(_I)
    lib.orc_accel_jerk(n, *[_p(a[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")], G, eps, hp, rp, cnt,
                       *[_p(o) for o in out[:6]], *sc, nthreads)
    return tuple(out)


def surface_density(x, y, nx, ny, x0, y0, sx, sy) -> np.ndarray:
    """Particle counts per x-y cell, shape (ny, nx), uint32: the surface-density
    maps of Section 3 (Fig. 7).  Cell index floor((x - x0) * sx) in float64."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape
    out = np.zeros((ny, nx), dtype=np.uint32)
    _load().orc_surface_density(x.size, _p(x), _p(y), int(nx), int(ny), float(x0), float(y0), float(sx),
                                float(sy), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def force_evals() -> int:
    return int(_load().orc_force_evals())


def reset_force_evals() -> None:
    _load().orc_reset_force_evals()
