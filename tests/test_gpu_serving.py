"""Serving on the GPU: requests that arrive while others run are batched
together; each result must equal the same request run alone (bitwise: under
the loop's batch plan a system's sums depend only on its own size and
precision) and float64 requests must track the oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_1803_01190_amd.serving import GpuBackend, Request, Scheduler

pytestmark = pytest.mark.gpu


def stream():
    rs = wl.request_stream(10, seed=5, rate=200.0, lo_log2=10, hi_log2=13, steps_lo=5, steps_hi=30,
                           fp64_fraction=0.3)
    return [Request(id=r["id"], t_arrive=r["t_arrive"], n=r["n"], steps=r["steps"], model=r["model"],
                    fp64=r["fp64"], seed=r["seed"]) for r in rs]


def test_mix_equals_alone_and_oracle(nb, ctx, orc):
    reqs = stream()
    be = GpuBackend(ctx, graph=True)
    st = Scheduler(be, hbm_budget=8 << 30, max_tick_steps=4).run(reqs)
    be.close()
    assert all(r.error is None for r in st.results), [r.error for r in st.results]
    s = st.summary()
    assert s["completed"] == len(reqs)
    # the requests really shared launches
    assert st.ticks < sum(r.steps for r in reqs)
    checked_oracle = False
    for r, q in zip(st.results, reqs):
        alone_be = GpuBackend(ctx, graph=False)
        alone = Scheduler(alone_be, hbm_budget=8 << 30, max_tick_steps=7).run([Request(**{**q.__dict__, "t_arrive": 0.0})])
        alone_be.close()
        a = alone.results[0]
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(r.state[k], a.state[k]), (q.id, k)
        if q.fp64 and not checked_oracle and q.n <= 4096:
            ic = wl.make(q.model, q.n, q.seed)
            h = wl.default_halo()
            halo = orc.Halo(h.v2, h.rc) if q.model == "disk" else None
            eps = 0.02 if q.model == "disk" else 0.01
            ref = orc.State(ic, eps=eps, halo=halo)
            ref.step_kdk(q.dt, q.steps)
            alt = orc.State(ic, eps=eps, halo=halo, reverse_j=True)
            alt.step_kdk(q.dt, q.steps)
            d_orc = max(np.max(np.abs(ref[k] - alt[k])) for k in ("x", "y", "z"))
            d_gpu = max(np.max(np.abs(r.state[k] - ref[k])) for k in ("x", "y", "z"))
            assert d_gpu <= 10 * d_orc + 1e-15, (d_gpu, d_orc)
            checked_oracle = True
    torch.cuda.synchronize()


def test_budget_queueing_on_gpu(nb, ctx):
    reqs = stream()[:6]
    be = GpuBackend(ctx)
    biggest = max(be.footprint(r) for r in reqs)
    st = Scheduler(be, hbm_budget=biggest + 1, max_tick_steps=4).run(reqs)
    be.close()
    assert all(r.error is None for r in st.results)
    # with room for about one request at a time, admissions are serial
    admits = sorted((r.t_admit, r.t_done) for r in st.results)
    for (a0, d0), (a1, d1) in zip(admits, admits[1:]):
        assert a1 >= a0
