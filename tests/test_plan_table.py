"""The tuned launch-plan table shipped with the package
(paper_1803_01190_amd/tuned_plans.json) holds only plans the library accepts
for their kernel class and precision, as documented for nbody_plan and the
NB_PLAN_* classes in include/nbody.h:
  * acceleration sum: R 1, 2 or 4; 128 or 256 lanes; split >= 1 (1 for
    float32); jsrc 0 or 1, or 2 to 5 (spatial order) for mixed with 256
    lanes and R 1 or 2;
  * potential pass: 256 lanes, R 1 or 2, jsrc 0 or 1;
  * acceleration-and-jerk sum: 256 lanes, R 1 or 2, jsrc 0, or 2 (spatial
    order) for mixed;
  * batch plans (mixed/batch, keyed by the largest system): 256 lanes, R 1 or
    2, split = source tiles per chunk >= 0 (0: whole systems), jsrc 0 or 2 to 5.
A bad entry would make load_plans fail on the GPU; this checks the file on
the host.  Keys are ceil(log2 n) of the size class."""
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1803_01190_amd", "tuned_plans.json")


def _ok(prec: str, cls: str, p: dict) -> bool:
    R, block, split, jsrc = p["R"], p["block"], p["split"], p["jsrc"]
    if cls == "batch":
        return (prec == "mixed" and block == 256 and R in (1, 2) and isinstance(split, int)
                and 0 <= split <= (1 << 20) and jsrc in (0, 2, 3, 4, 5))
    if not (isinstance(split, int) and 1 <= split <= 1024):
        return False
    if cls == "jerk":
        return block == 256 and R in (1, 2) and (jsrc == 0 or (jsrc == 2 and prec == "mixed"))
    if cls == "potential":
        return block == 256 and R in (1, 2) and jsrc in (0, 1)
    if jsrc in (2, 3, 4, 5):
        return prec == "mixed" and block == 256 and R in (1, 2)
    if prec == "fp32" and split != 1:
        return False
    return block in (128, 256) and R in (1, 2, 4) and jsrc in (0, 1)


def test_plan_table_entries_valid():
    with open(TABLE) as f:
        table = json.load(f)
    assert set(table) == {"gfx950"}
    n_plans = 0
    for key, sizes in table["gfx950"].items():
        prec, _, cls = key.partition("/")
        assert prec in ("fp64", "mixed", "fp32"), key
        assert cls in ("", "potential", "jerk", "batch"), key
        for log2n, plan in sizes.items():
            assert 0 <= int(log2n) <= 31, (key, log2n)
            assert set(plan) == {"R", "block", "split", "jsrc"}, (key, log2n, plan)
            assert _ok(prec, cls or "accel", plan), (key, log2n, plan)
            n_plans += 1
    assert n_plans > 0


def test_plan_table_covers_headline_sizes():
    # every precision has a pinned acceleration plan for N = 2^17 .. 2^20
    with open(TABLE) as f:
        t = json.load(f)["gfx950"]
    for prec in ("fp64", "mixed", "fp32"):
        for log2n in range(17, 21):
            assert str(log2n) in t[prec], (prec, log2n)


def test_plan_rule_rejects_known_bad_plans():
    # the rule itself: each documented restriction rejects a plan that breaks it
    good = {"R": 2, "block": 256, "split": 4, "jsrc": 0}
    assert _ok("fp64", "accel", good)
    bad = [
        ("fp64", "accel", dict(good, jsrc=3)),
        ("fp32", "accel", dict(good, jsrc=2)),
        ("mixed", "accel", dict(good, R=4, jsrc=3)),
        ("mixed", "accel", dict(good, block=128, jsrc=2)),
        ("mixed", "accel", dict(good, jsrc=6)),
        ("mixed", "jerk", dict(good, jsrc=4)),
        ("mixed", "jerk", dict(good, jsrc=5)),
        ("mixed", "batch", dict(good, jsrc=6)),
        ("fp32", "accel", dict(good, split=2)),
        ("fp64", "potential", dict(good, jsrc=2)),
        ("fp64", "potential", dict(good, block=128)),
        ("fp64", "jerk", dict(good, jsrc=1)),
        ("fp64", "jerk", dict(good, jsrc=2)),
        ("mixed", "jerk", dict(good, jsrc=3)),
        ("fp64", "jerk", dict(good, R=4)),
        ("fp64", "accel", dict(good, split=0)),
        ("mixed", "batch", dict(good, jsrc=1)),
        ("mixed", "batch", dict(good, R=4)),
        ("mixed", "batch", dict(good, block=128)),
        ("fp64", "batch", good),
    ]
    assert _ok("mixed", "batch", dict(good, split=0, jsrc=3))
    for prec, cls, p in bad:
        assert not _ok(prec, cls, p), (prec, cls, p)
