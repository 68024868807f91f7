"""CPU tests of the continuous-batching scheduler with a fake backend and a
virtual clock: admission by footprint, FIFO order, slot limits, failure
isolation and latency accounting (no GPU involved)."""
import pytest

from paper_1803_01190_amd.serving import Backend, Request, Result, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend(Backend):
    """Each step of the batch costs 1e-9 s per pair interaction of the
    active systems (virtual time); records what the scheduler asked."""

    def __init__(self, clock, fail_step=(), fail_admit=()):
        self.clock = clock
        self.live = {}
        self.steps_done = {}
        self.used = 0
        self.max_used = 0
        self.max_active = 0
        self.admit_order = []
        self.fail_step = set(fail_step)
        self.fail_admit = set(fail_admit)
        self.batches = []

    def footprint(self, req):
        return 80 * req.n

    def admit(self, req):
        if req.id in self.fail_admit:
            raise RuntimeError("injected admit failure")
        self.live[req.id] = req
        self.steps_done[req.id] = 0
        self.used += self.footprint(req)
        self.max_used = max(self.max_used, self.used)
        self.max_active = max(self.max_active, len(self.live))
        self.admit_order.append(req.id)
        return req.id

    def step(self, handles, nsteps):
        self.batches.append(sorted(handles))
        self.clock.t += 1e-9 * nsteps * sum(self.live[h].n ** 2 for h in handles)
        fails = {}
        for h in handles:
            if h in self.fail_step:
                fails[h] = "injected step failure"
            else:
                self.steps_done[h] += nsteps
        return fails

    def finish(self, h):
        r = self.live.pop(h)
        self.used -= self.footprint(r)
        return Result(r.id, r.n, r.steps, "mixed", r.t_arrive, state={"steps": self.steps_done[h]})

    def drop(self, h):
        r = self.live.pop(h)
        self.used -= self.footprint(r)


def reqs(specs):
    return [Request(id=i, t_arrive=t, n=n, steps=s) for i, (t, n, s) in enumerate(specs)]


def test_every_request_completes_with_its_step_count():
    clk = Clock()
    be = FakeBackend(clk)
    rs = reqs([(0.0, 1000, 10), (0.001, 2000, 25), (0.002, 500, 7), (0.5, 3000, 40)])
    st = Scheduler(be, hbm_budget=10**9, clock=clk, sleep=clk.sleep, max_tick_steps=5).run(rs)
    assert [r.id for r in st.results] == [0, 1, 2, 3]
    for r, q in zip(st.results, rs):
        assert r.error is None and r.state["steps"] == q.steps
        assert r.t_admit >= q.t_arrive and r.t_done >= r.t_admit
    s = st.summary()
    assert s["completed"] == 4 and s["latency_s"]["p50"] is not None
    assert s["latency_s"]["p99"] >= s["latency_s"]["p50"]


def test_budget_below_footprint_rejects_only_that_request():
    clk = Clock()
    be = FakeBackend(clk)
    rs = reqs([(0.0, 100, 5), (0.0, 10**6, 5), (0.0, 200, 5)])
    st = Scheduler(be, hbm_budget=80 * 1000, clock=clk, sleep=clk.sleep).run(rs)
    assert st.results[1].error and "exceeds" in st.results[1].error
    assert st.results[0].error is None and st.results[2].error is None


def test_full_budget_queues_fifo_and_never_overcommits():
    clk = Clock()
    be = FakeBackend(clk)
    # each needs 80 KB; budget fits two at a time
    rs = reqs([(0.0, 1000, 10), (0.0, 1000, 30), (0.0, 1000, 5), (0.0, 1000, 5), (0.0, 1000, 5)])
    st = Scheduler(be, hbm_budget=80 * 2000, clock=clk, sleep=clk.sleep).run(rs)
    assert all(r.error is None for r in st.results)
    assert be.max_used <= 80 * 2000 and be.max_active == 2
    assert be.admit_order == [0, 1, 2, 3, 4]
    # request 2 is admitted when request 0 retires, while request 1 still runs
    assert st.results[2].t_admit == pytest.approx(st.results[0].t_done)
    assert st.results[2].t_admit < st.results[1].t_done


def test_slot_limit():
    clk = Clock()
    be = FakeBackend(clk)
    rs = reqs([(0.0, 10, 3)] * 1 + [(0.0, 10, 3) for _ in range(9)])
    st = Scheduler(be, hbm_budget=10**9, max_slots=4, clock=clk, sleep=clk.sleep).run(rs)
    assert be.max_active == 4 and all(r.error is None for r in st.results)


def test_late_arrival_joins_running_batch():
    clk = Clock()
    be = FakeBackend(clk)
    # a long request is running when a short one arrives: the short one is
    # admitted at the next tick and shares the launches, not queued behind it
    rs = reqs([(0.0, 20000, 200), (0.05, 1000, 10)])
    st = Scheduler(be, hbm_budget=10**9, max_tick_steps=10, clock=clk, sleep=clk.sleep).run(rs)
    assert any(b == [0, 1] for b in be.batches)
    assert st.results[1].t_done < st.results[0].t_done


def test_failure_isolation():
    clk = Clock()
    be = FakeBackend(clk, fail_step={1}, fail_admit={3})
    rs = reqs([(0.0, 500, 10), (0.0, 500, 10), (0.0, 500, 10), (0.0, 500, 10)])
    st = Scheduler(be, hbm_budget=10**9, clock=clk, sleep=clk.sleep).run(rs)
    assert st.results[1].error == "injected step failure"
    assert st.results[3].error.startswith("admit failed")
    assert st.results[0].error is None and st.results[2].error is None
    assert st.results[0].state["steps"] == 10 and be.used == 0


def test_idle_gap_sleeps_until_next_arrival():
    clk = Clock()
    be = FakeBackend(clk)
    rs = reqs([(0.0, 100, 2), (5.0, 100, 2)])
    st = Scheduler(be, hbm_budget=10**9, clock=clk, sleep=clk.sleep).run(rs)
    assert st.results[1].t_admit >= 5.0 and st.results[1].latency < 1.0
