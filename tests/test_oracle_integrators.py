"""Pins for the oracle's time integrators.

KDK leapfrog, Eqs. (5)-(7) of Section 1 (one force evaluation per step), and
the fourth-order scheme the abstract names, read as the triple-jump
composition of the leapfrog step.  Pinned by exact free motion, the exact
discrete solution of the leapfrog map on a harmonic potential, Kepler's
equation with measured convergence orders, exact conservation of P and L
up to round-off, time reversibility and a degenerate composition.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_yoshida_weights(orc):
    w1, w0 = orc.YOSHIDA_W1, orc.YOSHIDA_W0
    assert abs(2 * w1 + w0 - 1) < 1e-15
    assert abs(2 * w1 ** 3 + w0 ** 3) < 1e-14
    assert abs(w1 - 1.3512071919596578) < 1e-15 and abs(w0 + 1.7024143839193155) < 1e-15


def test_free_particle(orc):
    ic = {"x": [1.0], "y": [2.0], "z": [3.0], "vx": [0.5], "vy": [-0.25], "vz": [0.125],
          "m": [1.0]}
    s = orc.State(ic, eps=0.1)
    s.step_kdk(0.125, 64)
    assert s["x"][0] == 1.0 + 8 * 0.5 and s["y"][0] == 2.0 - 8 * 0.25
    assert s["vx"][0] == 0.5 and s["ax"][0] == 0.0


def test_leapfrog_harmonic_exact_map(orc):
    # A particle near the centre of the cored halo moves in a harmonic
    # potential with w^2 = V_inf^2 / (3 rc^2).  The KDK map for x'' = -w^2 x
    # is linear with cos(theta) = 1 - w^2 dt^2 / 2; starting from rest at x0,
    # x_n = x0 cos(n theta) exactly.  A full kick in place of a half kick, or
    # a drift with the wrong velocity, changes theta.
    v2, rc = 3.0, 1.0
    w2 = v2 / (3 * rc * rc)
    x0, dt, n = 1e-7, 0.05, 400
    ic = {"x": [x0], "y": [0.0], "z": [0.0], "vx": [0.0], "vy": [0.0], "vz": [0.0], "m": [1.0]}
    s = orc.State(ic, halo=orc.Halo(v2, rc))
    s.step_kdk(dt, n)
    th = math.acos(1 - w2 * dt * dt / 2)
    assert abs(s["x"][0] / (x0 * math.cos(n * th)) - 1) < 1e-9
    # velocity at integer steps: v_n = -x0 sin(n theta) sin(theta) / dt
    assert abs(s["vx"][0] / (-x0 * math.sin(n * th) * math.sin(th) / dt) - 1) < 1e-9


def _kepler_error(orc, dt_count, scheme):
    g = json.load(open(os.path.join(GOLD, "kepler_e05.json")))
    T = g["period"]
    s = orc.State(wl.kepler_pair(), eps=0.0)
    t_end = 0.3 * T
    if scheme == "kdk":
        s.step_kdk(t_end / dt_count, dt_count)
    else:
        s.step_o4(t_end / dt_count, dt_count)
    rx = s["x"][1] - s["x"][0]
    ry = s["y"][1] - s["y"][0]
    ex, ey = wl.kepler_relative_position(t_end)
    dE = abs(s.diag()["E"] - g["E"])
    return math.hypot(rx - ex, ry - ey), dE


def test_kepler_second_order(orc):
    e1, E1 = _kepler_error(orc, 400, "kdk")
    e2, E2 = _kepler_error(orc, 800, "kdk")
    assert 1.8 < math.log2(e1 / e2) < 2.2
    assert 1.8 < math.log2(E1 / E2) < 2.2
    assert e2 < 1e-3


def test_kepler_fourth_order(orc):
    e1, _ = _kepler_error(orc, 200, "o4")
    e2, _ = _kepler_error(orc, 400, "o4")
    assert 3.6 < math.log2(e1 / e2) < 4.4
    assert e2 < 1e-6


def test_kepler_energy_and_lz(orc):
    g = json.load(open(os.path.join(GOLD, "kepler_e05.json")))
    s = orc.State(wl.kepler_pair(), eps=0.0)
    d0 = s.diag()
    assert abs(d0["E"] - g["E"]) < 1e-15 and abs(d0["Lz"] - g["Lz"]) < 1e-15
    s.step_kdk(g["period"] / 2000, 2000)
    d1 = s.diag()
    assert abs(d1["Lz"] - g["Lz"]) < 1e-15
    assert abs(d1["E"] / g["E"] - 1) < 1e-4


@pytest.mark.parametrize("scheme", ["kdk", "o4"])
def test_momentum_angular_momentum_roundoff(orc, scheme):
    p = wl.plummer(256, 12)
    s = orc.State(p, eps=0.01)
    d0 = s.diag()
    if scheme == "kdk":
        s.step_kdk(1e-3, 60)
    else:
        s.step_o4(1e-3, 20)
    d1 = s.diag()
    pscale = np.sum(p["m"] * np.sqrt(p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2))
    r = np.sqrt(p["x"] ** 2 + p["y"] ** 2 + p["z"] ** 2)
    lscale = np.sum(p["m"] * r * np.sqrt(p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2))
    for k in ("Px", "Py", "Pz"):
        assert abs(d1[k] - d0[k]) < 1e-14 * pscale
    for k in ("Lx", "Ly", "Lz"):
        assert abs(d1[k] - d0[k]) < 1e-13 * lscale
    assert abs(d1["E"] / d0["E"] - 1) < 1e-4


def test_time_reversibility(orc):
    p = wl.plummer(128, 13)
    s = orc.State(p, eps=0.02)
    x0 = s["x"].copy()
    v0 = s["vy"].copy()
    s.step_kdk(1e-3, 50)
    s.step_kdk(-1e-3, 50)
    assert np.max(np.abs(s["x"] - x0)) < 1e-13
    assert np.max(np.abs(s["vy"] - v0)) < 1e-12
    s.step_o4(2e-3, 10)
    s.step_o4(-2e-3, 10)
    assert np.max(np.abs(s["x"] - x0)) < 1e-13


def test_paper_form_matches_half_kick_form(orc):
    # Eqs. (5)-(7) rearranged: (v + v~)/2 = v + dt a / 2, so the two forms
    # differ only by rounding
    p = wl.plummer(200, 14)
    a = orc.State(p, eps=0.01)
    b = orc.State(p, eps=0.01)
    a.step_kdk(1e-3, 20, paper_form=False)
    b.step_kdk(1e-3, 20, paper_form=True)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-14 * np.max(np.abs(a[k]))
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-13 * np.max(np.abs(a[k]))


def test_one_force_evaluation_per_step(orc):
    p = wl.plummer(64, 15)
    s = orc.State(p, eps=0.01)
    orc.reset_force_evals()
    s.step_kdk(1e-3, 7)
    assert orc.force_evals() == 7
    orc.reset_force_evals()
    s.step_o4(1e-3, 5)
    assert orc.force_evals() == 15


def test_degenerate_composition(orc):
    # with weights (1/2, 0) the middle substep is the identity, so the
    # composition is exactly two leapfrog steps of dt/2
    p = wl.plummer(100, 16)
    a = orc.State(p, eps=0.01)
    b = orc.State(p, eps=0.01)
    a.step_o4(2e-3, 3, w1=0.5, w0=0.0)
    b.step_kdk(1e-3, 6)
    for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az"):
        assert np.array_equal(a[k], b[k]), k


def test_halo_breaks_momentum_not_lz(orc):
    # an external spherical field exerts a torque-free but non-zero net force
    d = wl.exp_disk(300, 17)
    s = orc.State(d, eps=0.02, halo=orc.Halo(**wl.default_halo().__dict__))
    d0 = s.diag()
    s.step_kdk(1e-3, 30)
    d1 = s.diag()
    assert abs(d1["Lz"] - d0["Lz"]) < 1e-13 * abs(d0["Lz"])
    assert abs(d1["E"] / d0["E"] - 1) < 1e-5
