"""Continuous-batching request loop over the batched C ABI.

Integration requests (initial conditions + number of KDK steps + precision)
arrive over time.  The scheduler admits them, first come first served, as
slots and the HBM budget allow; all admitted systems advance together in one
batched persistent launch per step (graph-replayed), so requests that arrive
while others run share the device; finished requests are retired at step
granularity and their slot and memory are released for the next arrival.

The scheduler is written against a small backend interface so that its
admission, ordering, failure isolation and latency accounting can be tested
on the CPU with a fake backend and a virtual clock; ``GpuBackend`` drives
libnbody.so.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

STATE_BYTES_PER_PARTICLE = 80  # x y z vx vy vz m ax ay az, float64
# Device bytes a request holds while active, per particle: its state twice
# (while the pack is rebuilt, the old pack, the new pack and newly admitted
# requests' own arrays are alive together), the batch's spatial order (keys,
# permutation, sorted positions and masses, tile boxes: about 64 B) and the
# diagnostics' potential (8 B); the partial sums of its source chunks are
# added per request (see GpuBackend.footprint).
ACTIVE_BYTES_PER_PARTICLE = 2 * STATE_BYTES_PER_PARTICLE + 64 + 8


@dataclass
class Request:
    id: int
    t_arrive: float
    n: int
    steps: int
    model: str = "plummer"
    fp64: bool = False
    seed: int = 0
    dt: float = 1e-3
    eps: Optional[float] = None
    ic: Optional[dict] = None  # initial conditions supplied with the request (else generated)


@dataclass
class Result:
    id: int
    n: int
    steps: int
    prec: str
    t_arrive: float
    t_admit: float = math.nan
    t_done: float = math.nan
    error: Optional[str] = None
    state: Optional[dict] = None
    diag: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class Backend:
    """Interface the scheduler drives."""

    def footprint(self, req: Request) -> int:  # device bytes while active
        raise NotImplementedError

    def admit(self, req: Request):  # -> handle; prepares state and a(t0)
        raise NotImplementedError

    def step(self, handles: list, nsteps: int) -> Dict[object, str]:
        """Advance every handle by nsteps; return {handle: error} for failures."""
        raise NotImplementedError

    def finish(self, handle) -> Result:
        """Result of a request that has run all its steps; releases it."""
        raise NotImplementedError

    def drop(self, handle) -> None:  # free without a result (after a failure)
        raise NotImplementedError


@dataclass
class Stats:
    results: List[Result] = field(default_factory=list)
    wall: float = 0.0
    ticks: int = 0
    steps_run: int = 0
    interactions: float = 0.0

    def summary(self) -> dict:
        done = [r for r in self.results if r.error is None]
        lat = sorted(r.latency for r in done)

        def pct(q):
            if not lat:
                return None
            k = (len(lat) - 1) * q
            lo, hi = math.floor(k), math.ceil(k)
            return lat[lo] + (lat[hi] - lat[lo]) * (k - lo)

        return {
            "completed": len(done),
            "failed": sum(1 for r in self.results if r.error is not None),
            "wall_s": self.wall,
            "requests_per_s": len(done) / self.wall if self.wall > 0 else None,
            "interactions_per_s": self.interactions / self.wall if self.wall > 0 else None,
            "latency_s": {"p50": pct(0.5), "p99": pct(0.99), "max": lat[-1] if lat else None},
            "ticks": self.ticks,
        }


class Scheduler:
    """FIFO admission by footprint, step-granular continuous batching.

    A request whose footprint exceeds the whole budget is rejected at once;
    otherwise the head of the queue waits until enough memory and a slot are
    free (no request overtakes an earlier one, so nothing starves).  Each tick
    advances all active requests by min(remaining steps, max_tick_steps).
    """

    def __init__(self, backend: Backend, hbm_budget: int, max_slots: int = 256,
                 max_tick_steps: int = 25, clock: Optional[Callable[[], float]] = None,
                 sleep: Optional[Callable[[float], None]] = None,
                 progress: Optional[Callable[[dict], None]] = None):
        self.b = backend
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_tick = max(1, int(max_tick_steps))
        self.clock = clock or time.monotonic
        self.sleep = sleep or time.sleep
        self.progress = progress  # called after every tick with counts and the time

    def run(self, requests: List[Request]) -> Stats:
        st = Stats()
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        pending = collections.deque(sorted(requests, key=lambda r: (r.t_arrive, r.id)))
        waiting: collections.deque = collections.deque()
        active: Dict[int, dict] = {}
        used = 0
        while pending or waiting or active:
            t = now()
            while pending and pending[0].t_arrive <= t:
                waiting.append(pending.popleft())
            # admission
            while waiting and len(active) < self.max_slots:
                r = waiting[0]
                fp = self.b.footprint(r)
                if fp > self.budget:
                    waiting.popleft()
                    st.results.append(Result(r.id, r.n, r.steps, "fp64" if r.fp64 else "mixed", r.t_arrive,
                                             t_admit=now(), t_done=now(),
                                             error=f"footprint {fp} B exceeds the HBM budget {self.budget} B"))
                    continue
                if used + fp > self.budget:
                    break
                waiting.popleft()
                try:
                    h = self.b.admit(r)
                except Exception as e:  # this request only
                    st.results.append(Result(r.id, r.n, r.steps, "fp64" if r.fp64 else "mixed", r.t_arrive,
                                             t_admit=now(), t_done=now(), error=f"admit failed: {e}"))
                    continue
                used += fp
                active[r.id] = {"req": r, "h": h, "left": r.steps, "fp": fp, "t_admit": now()}
            if not active:
                if pending:
                    dt = pending[0].t_arrive - now()
                    if dt > 0:
                        self.sleep(dt)
                continue
            k = min(min(a["left"] for a in active.values()), self.max_tick)
            fails: Dict[object, str] = {}
            if k > 0:
                handles = [a["h"] for a in active.values()]
                try:
                    fails = self.b.step(handles, k)
                except Exception as e:  # a failure of the shared launch fails every active request
                    fails = {a["h"]: f"step failed: {e}" for a in active.values()}
                st.ticks += 1
                st.steps_run += k
            for rid in list(active):
                a = active[rid]
                r = a["req"]
                if a["h"] in fails:
                    self.b.drop(a["h"])
                    used -= a["fp"]
                    del active[rid]
                    st.results.append(Result(r.id, r.n, r.steps, "fp64" if r.fp64 else "mixed", r.t_arrive,
                                             t_admit=a["t_admit"], t_done=now(), error=fails[a["h"]]))
                    continue
                a["left"] -= k
                if k > 0:
                    st.interactions += float(k) * float(r.n) * float(r.n)
                if a["left"] <= 0:
                    res = self.b.finish(a["h"])
                    res.t_arrive, res.t_admit, res.t_done = r.t_arrive, a["t_admit"], now()
                    st.results.append(res)
                    used -= a["fp"]
                    del active[rid]
            if self.progress is not None:
                self.progress({"t": now(), "active": len(active), "waiting": len(waiting), "pending": len(pending),
                               "done": len(st.results), "used_bytes": used})
        st.wall = now()
        st.results.sort(key=lambda r: r.id)
        return st


# ---------------------------------------------------------------------------
class GpuBackend(Backend):
    """Drives libnbody.so: active requests live packed back to back in one set
    of device arrays and one batch.  Whenever the set of active requests
    changes, the pack is rebuilt with device-to-device copies on the loop's
    stream and the batch is re-laid out for the new set with
    ``nbody_batch_reset`` (its device tables are reused and refilled by
    stream-ordered copies; nothing synchronises the device).  Between changes,
    steps replay a HIP graph captured for the current set (``graph``)."""

    def __init__(self, ctx, device="cuda", graph: bool = True, keep_state: bool = True,
                 diagnostics: bool = True, plan: Optional[dict] = None):
        import torch

        from . import nbody as nb
        import workloads as wl

        self.torch, self.nb, self.wl = torch, nb, wl
        self.ctx = ctx
        self.device = device
        self.graph = graph
        self.keep_state = keep_state
        self.diagnostics = diagnostics
        self.halo = wl.default_halo()
        # the batch plan of the loop: the one pinned for systems up to 2^20,
        # else the library's default
        self.plan = dict(plan) if plan is not None else nb.nbody_plan_get(ctx, nb.NB_MIXED | nb.NB_PLAN_BATCH, 1 << 20)
        # all device work of the loop goes to one non-blocking stream (default
        # priority)
        self.stream = torch.cuda.Stream()
        self.live: Dict[int, dict] = {}   # handle -> {req, sys (own arrays or view), prm}
        self.order: List[int] = []        # handles in pack order
        self.pack = None                  # packed System
        self.batch = None
        self.dirty = True

    def _chunks(self, n: int, fp32: bool = False) -> int:
        """Source chunks of an n-particle system under the loop's batch plan."""
        c = int(self.plan["split"])
        return 1 if (fp32 or c == 0) else max(1, -(-int(n) // (256 * c)))

    def footprint(self, req: Request) -> int:
        n = int(req.n)
        k = self._chunks(n)
        return ACTIVE_BYTES_PER_PARTICLE * n + (32 * k * n if k > 1 else 0)

    def _params(self, req: Request):
        nb, h = self.nb, self.halo
        disk = req.model == "disk"
        eps = req.eps if req.eps is not None else (0.02 if disk else 0.01)
        return nb.Params(G=1.0, eps=eps, prec=nb.NB_FP64 if req.fp64 else nb.NB_MIXED, halo=disk,
                         halo_v2=h.v2 if disk else 0.0, halo_rc=h.rc if disk else 0.0)

    def _alone_plan(self, prm, n: int) -> dict:
        """The single-system plan that gives this system's sums bitwise as the
        batch does (its chunk count; spatial order for NB_MIXED systems when
        the batch plan uses it)."""
        nb = self.nb
        return {"R": int(self.plan["R"]), "block": 256, "split": self._chunks(n, prm.prec == nb.NB_FP32),
                "jsrc": int(self.plan["jsrc"]) if prm.prec == nb.NB_MIXED else 0}

    def admit(self, req: Request):
        nb = self.nb
        ic = req.ic if req.ic is not None else self.wl.make(req.model, req.n, req.seed)
        with self.torch.cuda.stream(self.stream):
            s = nb.System.from_arrays(ic, device=self.device)
        prm = self._params(req)
        # a(t0) under the plan the batch takes for this system, which gives the
        # bits the batched kernels give
        nb.nbody_plan_set(self.ctx, prm.prec, req.n, self._alone_plan(prm, req.n))
        try:
            nb.nbody_accel(self.ctx, s, prm, stream=self.stream)
        finally:
            nb.nbody_plan_set(self.ctx, prm.prec, req.n, None)
        h = req.id
        self.live[h] = {"req": req, "sys": s, "prm": prm}
        self.dirty = True
        return h

    def _repack(self):
        nb, torch = self.nb, self.torch
        self.order = sorted(self.live)
        ns = [self.live[h]["req"].n for h in self.order]
        off = [0]
        for n in ns:
            off.append(off[-1] + n)
        with torch.cuda.stream(self.stream):
            pack = nb.System(off[-1], device=self.device)
            for k, h in enumerate(self.order):
                src = self.live[h]["sys"]
                for f in nb.FIELDS:
                    pack.t[f][off[k]:off[k + 1]].copy_(src.t[f])
        for k, h in enumerate(self.order):
            view = nb.System(0, device=self.device)
            view.n = ns[k]
            view.t = {f: pack.t[f][off[k]:off[k + 1]] for f in nb.FIELDS}
            view.t["phi"] = None
            self.live[h]["sys"] = view
        prms = [self.live[h]["prm"] for h in self.order]
        dts = [self.live[h]["req"].dt for h in self.order]
        if self.batch is None:
            self.batch = nb.nbody_batch_create(self.ctx, off, prms, dts,
                                               flags=nb.NB_BATCH_GRAPH if self.graph else 0)
            nb.nbody_batch_set_plan(self.ctx, self.batch, self.plan)
        else:
            nb.nbody_batch_reset(self.ctx, self.batch, off, prms, dts, stream=self.stream)
        self.pack = pack
        self.dirty = False

    def step(self, handles, nsteps):
        if self.dirty:
            self._repack()
        self.nb.nbody_step_kdk_batched(self.ctx, self.batch, self.pack, nsteps, stream=self.stream)
        return {}

    def _release(self, handle):
        del self.live[handle]
        self.dirty = True
        if not self.live:
            self.pack = None

    def finish(self, handle) -> Result:
        nb = self.nb
        e = self.live[handle]
        req, s, prm = e["req"], e["sys"], e["prm"]
        d = nb.diag_dict(nb.nbody_diag(self.ctx, s, prm, stream=self.stream)) if self.diagnostics else None
        if self.keep_state:
            self.stream.synchronize()
        state = s.numpy() if self.keep_state else None
        res = Result(req.id, req.n, req.steps, "fp64" if req.fp64 else "mixed", req.t_arrive, state=state, diag=d)
        if d is not None and not all(math.isfinite(v) for v in d.values()):
            res.error = "non-finite state"
        self._release(handle)
        return res

    def drop(self, handle) -> None:
        self._release(handle)

    def close(self):
        self.stream.synchronize()
        if self.batch is not None:
            self.nb.nbody_batch_destroy(self.ctx, self.batch)
            self.batch = None
