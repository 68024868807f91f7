"""Thin ctypes binding of the C ABI in include/nbody.h.

Argument marshalling only: every step of the force sum, the integrators and
the diagnostics runs in the HIP kernels of libnbody.so.  PyTorch provides the
device memory (float64 CUDA tensors) and the stream handle.  There is no CPU
fallback: if the library is missing, importing this module raises.

The functions carry the C names (``nbody_accel``, ``nbody_step_kdk`` ...);
``System``, ``Params`` and ``Context`` are small conveniences around them.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")

NB_OK, NB_EINVAL, NB_ENOMEM, NB_EHIP, NB_ENOTSUP = 0, -1, -2, -3, -4
NB_FP64, NB_MIXED, NB_FP32 = 0, 1, 2
NB_BATCH_GRAPH = 1
PREC = {"fp64": NB_FP64, "mixed": NB_MIXED, "fp32": NB_FP32}
NB_PLAN_ACCEL, NB_PLAN_POTENTIAL, NB_PLAN_JERK, NB_PLAN_BATCH = 0x000, 0x100, 0x200, 0x300
PLAN_CLASS = {"accel": NB_PLAN_ACCEL, "potential": NB_PLAN_POTENTIAL, "jerk": NB_PLAN_JERK, "batch": NB_PLAN_BATCH}
FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az")


class NBodyError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nbody error {status}: {msg}")
        self.status = status


class c_sys(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                          ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az", "phi")]


class c_params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("eps", ctypes.c_double), ("prec", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("halo_v2", ctypes.c_double), ("halo_rc", ctypes.c_double)]


class c_plan(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("block", ctypes.c_int32), ("split", ctypes.c_int32),
                ("jsrc", ctypes.c_int32)]

    def as_dict(self):
        return {"R": self.R, "block": self.block, "split": self.split, "jsrc": self.jsrc}


class c_profile(ctypes.Structure):
    _fields_ = [("accel_launches", ctypes.c_int64), ("accel_ms", ctypes.c_double),
                ("interactions", ctypes.c_int64), ("update_launches", ctypes.c_int64),
                ("update_ms", ctypes.c_double)]


DIAG_KEYS = ("K", "W", "Wext", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "Cx", "Cy", "Cz", "M")


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1803_01190_amd/build.py "
                           "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I64, I32, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    S, PR = ctypes.POINTER(c_sys), ctypes.POINTER(c_params)
    sig = {
        "nbody_ctx_create": ([ctypes.c_int, ctypes.POINTER(P)]),
        "nbody_ctx_destroy": ([P]),
        "nbody_accel": ([P, S, PR, V]),
        "nbody_accel_rows": ([P, S, PR, I64, I64, V]),
        "nbody_accel_static": ([P, S, PR, V]),
        "nbody_accel_order_rows": ([P, S, PR, I64, I64, V]),
        "nbody_step_kdk": ([P, S, PR, D, I64, V]),
        "nbody_step_o4": ([P, S, PR, D, I64, V]),
        "nbody_diag": ([P, S, PR, V, V]),
        "nbody_accel_jerk": ([P, S, V, V, V, PR, V]),
        "nbody_step_hermite": ([P, S, V, V, V, PR, D, I64, V]),
        "nbody_step_rk4": ([P, S, PR, D, I64, V]),
        "nbody_surface_density": ([P, S, I32, I32, D, D, D, D, V, V]),
        "nbody_spatial_order": ([P, S, V, V, V]),
        "nbody_batch_create": ([P, I32, ctypes.POINTER(I64), PR, ctypes.POINTER(D), ctypes.c_uint32,
                                ctypes.POINTER(P)]),
        "nbody_batch_destroy": ([P, P]),
        "nbody_batch_reset": ([P, P, I32, ctypes.POINTER(I64), PR, ctypes.POINTER(D), V]),
        "nbody_batch_get_plan": ([P, P, ctypes.POINTER(c_plan)]),
        "nbody_batch_set_plan": ([P, P, ctypes.POINTER(c_plan)]),
        "nbody_batch_system_plan": ([P, P, I32, ctypes.POINTER(c_plan)]),
        "nbody_accel_batched": ([P, P, S, V]),
        "nbody_step_kdk_batched": ([P, P, S, I64, V]),
        "nbody_step_o4_batched": ([P, P, S, I64, V]),
        "nbody_diag_batched": ([P, P, S, V, V]),
        "nbody_plan_get": ([P, I32, I64, ctypes.POINTER(c_plan)]),
        "nbody_plan_set": ([P, I32, I64, ctypes.POINTER(c_plan)]),
        "nbody_autotune": ([P, I32, I64, D, ctypes.POINTER(c_plan)]),
        "nbody_autotune_sys": ([P, I32, S, PR, D, ctypes.POINTER(c_plan)]),
        "nbody_batch_autotune": ([P, P, S, D, ctypes.POINTER(c_plan)]),
        "nbody_profile_enable": ([P, ctypes.c_int]),
        "nbody_profile_read": ([P, ctypes.POINTER(c_profile)]),
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.nbody_last_error.argtypes = [P]
    lib.nbody_last_error.restype = ctypes.c_char_p
    lib.nbody_version.restype = ctypes.c_char_p
    return lib


_lib = _load()


def version() -> str:
    return _lib.nbody_version().decode()


def _check(ctx, status: int):
    if status != NB_OK:
        msg = _lib.nbody_last_error(ctx).decode() if ctx else ""
        raise NBodyError(status, msg)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


@dataclass
class Params:
    G: float = 1.0
    eps: float = 0.0
    prec: int = NB_FP64
    halo: bool = False
    halo_v2: float = 0.0
    halo_rc: float = 0.0

    def c(self) -> c_params:
        return c_params(float(self.G), float(self.eps), int(self.prec), int(bool(self.halo)),
                        float(self.halo_v2), float(self.halo_rc))


class System:
    """Float64 structure-of-arrays particle state on a CUDA (HIP) device."""

    def __init__(self, n: int, device="cuda", with_phi: bool = False):
        self.n = int(n)
        self.t = {k: torch.zeros(self.n, dtype=torch.float64, device=device) for k in FIELDS}
        self.t["phi"] = torch.zeros(self.n, dtype=torch.float64, device=device) if with_phi else None

    @classmethod
    def from_arrays(cls, d: dict, device="cuda", with_phi: bool = False) -> "System":
        n = len(d["x"])
        s = cls(n, device, with_phi)
        for k in ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az"):
            if k in d:
                s.t[k].copy_(torch.as_tensor(d[k], dtype=torch.float64))
        if "jx" in d:
            for k in ("jx", "jy", "jz"):
                s.jerk(k).copy_(torch.as_tensor(d[k], dtype=torch.float64))
        return s

    def jerk(self, k: str) -> torch.Tensor:
        """The jerk array k (jx, jy or jz) of the Hermite scheme, allocated
        on first use."""
        if self.t.get(k) is None:
            self.t[k] = torch.zeros(self.n, dtype=torch.float64, device=self.t["x"].device)
        return self.t[k]

    def jerk_ptrs(self):
        return [ctypes.c_void_p(self.jerk(k).data_ptr() if self.n > 0 else None) for k in ("jx", "jy", "jz")]

    def __getitem__(self, k):
        return self.t[k]

    def numpy(self) -> dict:
        return {k: v.cpu().numpy() for k, v in self.t.items() if v is not None}

    def c(self) -> c_sys:
        t = self.t
        for k, v in t.items():
            if v is not None:
                assert v.dtype == torch.float64 and v.is_contiguous() and v.numel() == self.n, k
        p = lambda k: t[k].data_ptr() if (t[k] is not None and self.n > 0) else None
        return c_sys(self.n, *[p(k) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az", "phi")])


# ---- the C entry points, same names ----------------------------------------

def nbody_ctx_create(device: int = 0):
    h = ctypes.c_void_p()
    st = _lib.nbody_ctx_create(int(device), ctypes.byref(h))
    if st != NB_OK:
        raise NBodyError(st, "context creation failed")
    return h


def nbody_ctx_destroy(ctx):
    _check(None, _lib.nbody_ctx_destroy(ctx))


def nbody_accel(ctx, sys: System, prm: Params, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_accel(ctx, ctypes.byref(cs), ctypes.byref(cp), _stream(stream)))


def nbody_accel_order_rows(ctx, sys: System, prm: Params, k0: int, k1: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_accel_order_rows(ctx, ctypes.byref(cs), ctypes.byref(cp), int(k0), int(k1),
                                            _stream(stream)))


def nbody_accel_static(ctx, sys: System, prm: Params, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_accel_static(ctx, ctypes.byref(cs), ctypes.byref(cp), _stream(stream)))


def nbody_accel_rows(ctx, sys: System, prm: Params, i0: int, i1: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_accel_rows(ctx, ctypes.byref(cs), ctypes.byref(cp), int(i0), int(i1),
                                      _stream(stream)))


def nbody_step_kdk(ctx, sys: System, prm: Params, dt: float, nsteps: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_step_kdk(ctx, ctypes.byref(cs), ctypes.byref(cp), float(dt), int(nsteps),
                                    _stream(stream)))


def nbody_step_o4(ctx, sys: System, prm: Params, dt: float, nsteps: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_step_o4(ctx, ctypes.byref(cs), ctypes.byref(cp), float(dt), int(nsteps),
                                   _stream(stream)))


def nbody_accel_jerk(ctx, sys: System, prm: Params, stream=None):
    """a and the jerk (into sys['jx'], ['jy'], ['jz']) at the current state."""
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_accel_jerk(ctx, ctypes.byref(cs), *sys.jerk_ptrs(), ctypes.byref(cp), _stream(stream)))


def nbody_step_hermite(ctx, sys: System, prm: Params, dt: float, nsteps: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_step_hermite(ctx, ctypes.byref(cs), *sys.jerk_ptrs(), ctypes.byref(cp), float(dt),
                                        int(nsteps), _stream(stream)))


def nbody_step_rk4(ctx, sys: System, prm: Params, dt: float, nsteps: int, stream=None):
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_step_rk4(ctx, ctypes.byref(cs), ctypes.byref(cp), float(dt), int(nsteps),
                                    _stream(stream)))


def nbody_diag(ctx, sys: System, prm: Params, out: torch.Tensor | None = None, stream=None):
    """Returns a float64 device tensor of 14 values (see DIAG_KEYS)."""
    if out is None:
        out = torch.empty(14, dtype=torch.float64, device=sys.t["x"].device)
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_diag(ctx, ctypes.byref(cs), ctypes.byref(cp), ctypes.c_void_p(out.data_ptr()),
                                _stream(stream)))
    return out


def nbody_surface_density(ctx, sys: System, nx: int, ny: int, x0: float, y0: float, sx: float, sy: float,
                          out: torch.Tensor | None = None, stream=None):
    """Counts of particles per x-y cell, an int32 device tensor of shape
    (ny, nx) holding the library's uint32 counts (n < 2^31)."""
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.int32, device=sys.t["x"].device)
    assert out.dtype == torch.int32 and out.is_contiguous() and out.numel() == nx * ny
    cs = sys.c()
    _check(ctx, _lib.nbody_surface_density(ctx, ctypes.byref(cs), int(nx), int(ny), float(x0), float(y0),
                                           float(sx), float(sy), ctypes.c_void_p(out.data_ptr()),
                                           _stream(stream)))
    return out


def nbody_spatial_order(ctx, sys: System, stream=None):
    """(perm, keys): the Morton order of the spatially ordered plans (jsrc 2 to 5) as device tensors
    (int32 permutation; the sorted uint64 keys held in an int64 tensor)."""
    dev = sys.t["x"].device
    perm = torch.empty(sys.n, dtype=torch.int32, device=dev)
    keys = torch.empty(sys.n, dtype=torch.int64, device=dev)
    cs = sys.c()
    _check(ctx, _lib.nbody_spatial_order(ctx, ctypes.byref(cs), ctypes.c_void_p(perm.data_ptr() if sys.n else None),
                                         ctypes.c_void_p(keys.data_ptr() if sys.n else None), _stream(stream)))
    return perm, keys


def diag_dict(t: torch.Tensor) -> dict:
    return dict(zip(DIAG_KEYS, t.cpu().tolist()))


def nbody_batch_create(ctx, off, prms, dts=None, flags: int = 0):
    B = len(off) - 1
    off_a = (ctypes.c_int64 * (B + 1))(*[int(v) for v in off])
    prm_a = (c_params * B)(*[p.c() for p in prms])
    dt_a = (ctypes.c_double * B)(*[float(v) for v in dts]) if dts is not None else None
    h = ctypes.c_void_p()
    _check(ctx, _lib.nbody_batch_create(ctx, B, off_a, prm_a, dt_a, int(flags), ctypes.byref(h)))
    return h


def nbody_batch_reset(ctx, batch, off, prms, dts=None, stream=None):
    B = len(off) - 1
    off_a = (ctypes.c_int64 * (B + 1))(*[int(v) for v in off])
    prm_a = (c_params * B)(*[p.c() for p in prms])
    dt_a = (ctypes.c_double * B)(*[float(v) for v in dts]) if dts is not None else None
    _check(ctx, _lib.nbody_batch_reset(ctx, batch, B, off_a, prm_a, dt_a, _stream(stream)))


def nbody_batch_destroy(ctx, batch):
    _check(ctx, _lib.nbody_batch_destroy(ctx, batch))


def nbody_batch_get_plan(ctx, batch) -> dict:
    p = c_plan()
    _check(ctx, _lib.nbody_batch_get_plan(ctx, batch, ctypes.byref(p)))
    return p.as_dict()


def nbody_batch_set_plan(ctx, batch, plan: dict):
    p = c_plan(int(plan["R"]), int(plan["block"]), int(plan["split"]), int(plan.get("jsrc", 0)))
    _check(ctx, _lib.nbody_batch_set_plan(ctx, batch, ctypes.byref(p)))


def nbody_batch_system_plan(ctx, batch, sys: int) -> dict:
    p = c_plan()
    _check(ctx, _lib.nbody_batch_system_plan(ctx, batch, int(sys), ctypes.byref(p)))
    return p.as_dict()


def nbody_accel_batched(ctx, batch, all_sys: System, stream=None):
    cs = all_sys.c()
    _check(ctx, _lib.nbody_accel_batched(ctx, batch, ctypes.byref(cs), _stream(stream)))


def nbody_step_kdk_batched(ctx, batch, all_sys: System, nsteps: int, stream=None):
    cs = all_sys.c()
    _check(ctx, _lib.nbody_step_kdk_batched(ctx, batch, ctypes.byref(cs), int(nsteps), _stream(stream)))


def nbody_step_o4_batched(ctx, batch, all_sys: System, nsteps: int, stream=None):
    cs = all_sys.c()
    _check(ctx, _lib.nbody_step_o4_batched(ctx, batch, ctypes.byref(cs), int(nsteps), _stream(stream)))


def nbody_diag_batched(ctx, batch, all_sys: System, B: int, out: torch.Tensor | None = None, stream=None):
    if out is None:
        out = torch.empty((B, 14), dtype=torch.float64, device=all_sys.t["x"].device)
    cs = all_sys.c()
    _check(ctx, _lib.nbody_diag_batched(ctx, batch, ctypes.byref(cs), ctypes.c_void_p(out.data_ptr()),
                                        _stream(stream)))
    return out


def nbody_plan_get(ctx, prec: int, n: int) -> dict:
    p = c_plan()
    _check(ctx, _lib.nbody_plan_get(ctx, int(prec), int(n), ctypes.byref(p)))
    return p.as_dict()


def nbody_plan_set(ctx, prec: int, n: int, plan: dict | None):
    """Pin ``plan`` for the size class of n; ``None`` removes the pin."""
    if plan is None:
        _check(ctx, _lib.nbody_plan_set(ctx, int(prec), int(n), None))
        return
    p = c_plan(int(plan["R"]), int(plan["block"]), int(plan["split"]), int(plan.get("jsrc", 0)))
    _check(ctx, _lib.nbody_plan_set(ctx, int(prec), int(n), ctypes.byref(p)))


TUNED_PLANS = os.path.join(_HERE, "tuned_plans.json")


def plan_code(key: str) -> int:
    """Precision-and-class code of a plan-cache key: "fp64" (the acceleration
    sum) or "fp64/potential", "mixed/jerk", ..."""
    prec, _, cls = key.partition("/")
    return PREC[prec] | PLAN_CLASS[cls or "accel"]


def read_plans(path: str = TUNED_PLANS, arch: str = "gfx950") -> dict:
    """{key: {log2n: plan}} from a plan-cache file (empty if absent); keys as
    in plan_code."""
    import json
    try:
        with open(path) as f:
            return json.load(f).get(arch, {})
    except (OSError, ValueError):
        return {}


def load_plans(ctx, path: str = TUNED_PLANS, arch: str = "gfx950") -> int:
    """Pin every plan of a plan-cache file; returns how many were pinned."""
    k = 0
    for key, table in read_plans(path, arch).items():
        for log2n, plan in table.items():
            nbody_plan_set(ctx, plan_code(key), 1 << int(log2n), plan)
            k += 1
    return k


def nbody_autotune(ctx, prec: int, n: int, budget_ms: float = 2000.0) -> dict:
    p = c_plan()
    _check(ctx, _lib.nbody_autotune(ctx, int(prec), int(n), float(budget_ms), ctypes.byref(p)))
    return p.as_dict()


def nbody_autotune_sys(ctx, prec: int, sys: System, prm: Params, budget_ms: float = 2000.0) -> dict:
    p = c_plan()
    cs, cp = sys.c(), prm.c()
    _check(ctx, _lib.nbody_autotune_sys(ctx, int(prec), ctypes.byref(cs), ctypes.byref(cp), float(budget_ms),
                                        ctypes.byref(p)))
    return p.as_dict()


def nbody_batch_autotune(ctx, batch, all_sys: System, budget_ms: float = 4000.0) -> dict:
    p = c_plan()
    cs = all_sys.c()
    _check(ctx, _lib.nbody_batch_autotune(ctx, batch, ctypes.byref(cs), float(budget_ms), ctypes.byref(p)))
    return p.as_dict()


def nbody_profile_enable(ctx, on: bool = True):
    _check(ctx, _lib.nbody_profile_enable(ctx, int(bool(on))))


def nbody_profile_read(ctx) -> dict:
    p = c_profile()
    _check(ctx, _lib.nbody_profile_read(ctx, ctypes.byref(p)))
    return {k: getattr(p, k) for k, _ in c_profile._fields_}


class Context:
    """Owns one library context on a device."""

    def __init__(self, device: int = 0):
        self.h = nbody_ctx_create(device)

    def close(self):
        if self.h:
            nbody_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
