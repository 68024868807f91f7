"""Pins of the force-error metrics every parity gate goes through
(oracle/metrics.py): hand-worked accelerations whose four measures are known
in closed form, including a target whose reference acceleration is zero and
one whose condition scale is zero.

The definitions pinned here are those of the conditioned and relative force
errors (eps_rms, eps_norm, eps_cond, eps_max) stated with force_errors.
NBODY_METRICS_SRC selects another copy of the module (the planted-mistake
tests load mutated copies through it)."""
import importlib.util
import math
import os

import numpy as np
import pytest


def _metrics():
    alt = os.environ.get("NBODY_METRICS_SRC")
    if not alt:
        from oracle import metrics
        return metrics
    spec = importlib.util.spec_from_file_location("_metrics_under_test", alt)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def fe():
    return _metrics().force_errors


# Four targets (columns).  Differences got - ref and their lengths:
#   0: ref (3, 4, 0), |ref| 5, diff (0, 0, 1), |d| 1, scale 10
#   1: ref (0, 0, 2), |ref| 2, diff 0,           |d| 0, scale 4
#   2: ref (1, 2, 2), |ref| 3, diff (2, 1, 2),   |d| 3, scale 6
#   3: ref 0,         |ref| 0, diff (0, 0.5, 0), |d| 0.5, scale 0
REF = np.array([[3.0, 0.0, 1.0, 0.0],
                [4.0, 0.0, 2.0, 0.0],
                [0.0, 2.0, 2.0, 0.0]])
DIFF = np.array([[0.0, 0.0, 2.0, 0.0],
                 [0.0, 0.0, 1.0, 0.5],
                 [1.0, 0.0, 2.0, 0.0]])
SCALE = np.array([10.0, 4.0, 6.0, 0.0])


def test_hand_worked(fe):
    e = fe(REF + DIFF, REF, SCALE)
    # relative errors of the targets with a nonzero reference: 1/5, 0, 3/3
    assert e["eps_rms"] == pytest.approx(math.sqrt((0.2 ** 2 + 0.0 + 1.0) / 3.0), rel=1e-15)
    # norms over every target: sqrt(1 + 9 + 0.25) / sqrt(25 + 4 + 9)
    assert e["eps_norm"] == pytest.approx(math.sqrt(10.25) / math.sqrt(38.0), rel=1e-15)
    # |d| / A over the targets with A > 0: 1/10, 0/4, 3/6
    assert e["eps_cond"] == pytest.approx(0.5, rel=1e-15)
    assert e["eps_max"] == pytest.approx(1.0, rel=1e-15)


def test_three_targets_square_layout(fe):
    # a 3 x 3 input: reducing over the wrong axis gives other numbers here
    # rather than an error
    ref = np.array([[1.0, 0.0, 0.0],
                    [0.0, 2.0, 0.0],
                    [0.0, 0.0, 4.0]])
    diff = np.array([[0.0, 0.0, 0.0],
                     [0.1, 0.0, 0.0],
                     [0.0, 0.0, 0.0]])
    e = fe(ref + diff, ref, np.array([1.0, 1.0, 1.0]))
    assert e["eps_rms"] == pytest.approx(math.sqrt(0.01 / 3.0), rel=1e-14)
    assert e["eps_norm"] == pytest.approx(0.1 / math.sqrt(21.0), rel=1e-14)
    assert e["eps_cond"] == pytest.approx(0.1, rel=1e-14)
    assert e["eps_max"] == pytest.approx(0.1, rel=1e-14)


def test_exact_and_zero_scale(fe):
    e = fe(REF, REF, SCALE)
    assert e == {"eps_rms": 0.0, "eps_norm": 0.0, "eps_cond": 0.0, "eps_max": 0.0}
    # no target with a positive condition scale: eps_cond is the largest |d|
    e = fe(REF + DIFF, REF, np.zeros(4))
    assert e["eps_cond"] == pytest.approx(3.0, rel=1e-15)


def test_single_bad_target_dominates_max_not_rms(fe):
    # 1000 targets, one with relative error 1e-3, the rest exact: eps_max and
    # eps_cond see it fully, eps_rms by sqrt(1/1000)
    k = 1000
    ref = np.zeros((3, k))
    ref[0] = 2.0
    got = ref.copy()
    got[0, 17] = 2.0 + 2e-3
    e = fe(got, ref, np.full(k, 4.0))
    assert e["eps_max"] == pytest.approx(1e-3, rel=1e-12)
    assert e["eps_cond"] == pytest.approx(5e-4, rel=1e-12)
    assert e["eps_rms"] == pytest.approx(1e-3 / math.sqrt(k), rel=1e-12)
    assert e["eps_norm"] == pytest.approx(2e-3 / (2.0 * math.sqrt(k)), rel=1e-12)
