"""Host logic of bench.py that decides what the JSON line reports, checked on
the CPU: the HBM traffic figure comes from the committed counter summary only
while the kernel sources and the launch plan are the ones it was measured on,
and the percentile helper the latency figures use."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record():
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as f:
        return json.load(f)


def test_traffic_reported_for_the_measured_sources_and_plan():
    rec = _record()
    if rec["kernel_hash"] != bench.kernel_hash():
        pytest.skip("kernel sources changed since the counters were taken: the bench reports traffic null")
    for prec, plan in rec["plans"].items():
        assert bench.load_traffic(prec, plan) == rec["per_launch_bytes"][prec]


def test_traffic_null_for_another_plan_or_source(monkeypatch):
    rec = _record()
    plan = dict(rec["plans"]["mixed"])
    other = dict(plan, split=plan["split"] * 2)
    assert bench.load_traffic("mixed", other) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.load_traffic("mixed", plan) is None


def test_traffic_covers_the_partial_sums_of_the_plan():
    # the mixed launch writes its split partial sums: 32 B per particle per
    # chunk at N = 2^20, all of which the measured bytes must include
    rec = _record()
    split = rec["plans"]["mixed"]["split"]
    assert rec["per_launch_bytes"]["mixed"] >= 32 * split * (1 << 20)


@pytest.mark.parametrize("xs,q,want", [([3.0], 0.5, 3.0), ([1.0, 2.0, 3.0, 4.0], 0.5, 2.5),
                                       ([4.0, 1.0, 3.0, 2.0], 0.0, 1.0), ([4.0, 1.0, 3.0, 2.0], 1.0, 4.0),
                                       ([0.0, 10.0], 0.99, 9.9)])
def test_percentile_interpolates_between_order_statistics(xs, q, want):
    assert bench.percentile(xs, q) == pytest.approx(want)
