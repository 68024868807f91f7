"""Pins for the oracle's other fourth-order schemes: the jerk (the time
derivative of Eqs. (1)-(2) along the motion), the fourth-order Hermite
scheme built on it, and classical fourth-order Runge-Kutta (Section 1
contrasts the leapfrog's one force evaluation per step with Runge-Kutta
schemes).

The jerk is pinned by central differences of the (separately pinned)
acceleration along the motion, the halo's jerk likewise on both sides of its
series branch point; the schemes by Kepler's equation with measured
convergence orders, round-off conservation of P, a circular orbit in the
halo, and their force-evaluation counts."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _moved(p, h):
    q = {k: np.asarray(v, dtype=np.float64) for k, v in p.items()}
    for c in "xyz":
        q[c] = q[c] + h * q["v" + c]
    return q


def test_jerk_is_time_derivative_of_accel(orc):
    p = wl.plummer(300, 21)
    eps, h = 0.01, 1e-5
    ax, ay, az, jx, jy, jz = orc.accel_jerk(p, 1.0, eps)
    a = orc.accel(p["x"], p["y"], p["z"], p["m"], 1.0, eps)
    scale = np.sqrt(np.mean(a[0] ** 2 + a[1] ** 2 + a[2] ** 2))
    for got, ref in zip((ax, ay, az), a[:3]):
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale
    qp, qm = _moved(p, h), _moved(p, -h)
    ap = orc.accel(qp["x"], qp["y"], qp["z"], p["m"], 1.0, eps)
    am = orc.accel(qm["x"], qm["y"], qm["z"], p["m"], 1.0, eps)
    jscale = np.sqrt(np.mean(jx ** 2 + jy ** 2 + jz ** 2))
    for got, c in zip((jx, jy, jz), range(3)):
        fd = (ap[c] - am[c]) / (2 * h)
        assert np.max(np.abs(got - fd)) <= 1e-6 * jscale


def test_jerk_two_body_closed_form(orc):
    # two bodies, r = (1, 0, 0) apart, relative velocity (0.3, 0.4, 0): with
    # R^2 = 1 + eps^2, the jerk on body 0 from body 1 (mass 1) is
    # v/R^3 - 3 (r.v) r / R^5 = (0.3/R^3 - 0.9/R^5, 0.4/R^3, 0)
    p = {"x": [0.0, 1.0], "y": [0.0, 0.0], "z": [0.0, 0.0], "vx": [0.0, 0.3], "vy": [0.0, 0.4],
         "vz": [0.0, 0.0], "m": [2.0, 1.0]}
    eps = 0.5
    R2 = 1 + eps * eps
    R3, R5 = R2 ** 1.5, R2 ** 2.5
    ax, ay, az, jx, jy, jz = orc.accel_jerk(p, 1.0, eps)
    assert abs(ax[0] - 1 / R3) < 1e-15 and abs(ax[1] + 2 / R3) < 1e-15
    assert abs(jx[0] - (0.3 / R3 - 0.9 / R5)) < 1e-15 and abs(jy[0] - 0.4 / R3) < 1e-15
    assert jz[0] == 0.0
    # equal and opposite, weighted by mass: m0 j0 + m1 j1 = 0
    assert abs(2 * jx[0] + 1 * jx[1]) < 1e-15 and abs(2 * jy[0] + jy[1]) < 1e-15


@pytest.mark.parametrize("r0", [0.05, 0.3, 0.49, 0.51, 1.7, 12.0])
def test_halo_jerk_along_motion(orc, r0):
    # one particle in the halo field alone; radius r0 straddles the series
    # branch point s = 1/2 (rc = 1)
    v2, rc = 1.3, 1.0
    d = np.array([0.6, -0.48, 0.64])
    d = d / np.linalg.norm(d)
    p = {"x": [r0 * d[0]], "y": [r0 * d[1]], "z": [r0 * d[2]], "vx": [0.3], "vy": [0.5], "vz": [-0.2],
         "m": [1.0]}
    halo = orc.Halo(v2, rc)
    ax, ay, az, jx, jy, jz = orc.accel_jerk(p, 1.0, 0.0, halo)
    hx, hy, hz = orc.halo_accel(p["x"], p["y"], p["z"], halo)
    assert (ax[0], ay[0], az[0]) == (hx[0], hy[0], hz[0])
    h = 1e-6 * max(r0, 0.1)
    qp, qm = _moved(p, h), _moved(p, -h)
    ap = orc.halo_accel(qp["x"], qp["y"], qp["z"], halo)
    am = orc.halo_accel(qm["x"], qm["y"], qm["z"], halo)
    js = math.sqrt(jx[0] ** 2 + jy[0] ** 2 + jz[0] ** 2)
    for got, c in zip((jx[0], jy[0], jz[0]), range(3)):
        fd = (ap[c][0] - am[c][0]) / (2 * h)
        assert abs(got - fd) <= 1e-7 * js, (r0, c, got, fd)


def _kepler_error(orc, count, scheme):
    g = json.load(open(os.path.join(GOLD, "kepler_e05.json")))
    s = orc.State(wl.kepler_pair(), eps=0.0)
    t_end = 0.3 * g["period"]
    getattr(s, "step_" + scheme)(t_end / count, count)
    ex, ey = wl.kepler_relative_position(t_end)
    err = math.hypot(s["x"][1] - s["x"][0] - ex, s["y"][1] - s["y"][0] - ey)
    return err, abs(s.diag()["E"] - g["E"])


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
def test_kepler_fourth_order(orc, scheme):
    e1, E1 = _kepler_error(orc, 200, scheme)
    e2, E2 = _kepler_error(orc, 400, scheme)
    assert 3.6 < math.log2(e1 / e2) < 4.4, (e1, e2)
    assert e2 < 1e-5


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
def test_momentum_roundoff(orc, scheme):
    p = wl.plummer(200, 22)
    s = orc.State(p, eps=0.01)
    d0 = s.diag()
    getattr(s, "step_" + scheme)(1e-3, 10)
    d1 = s.diag()
    pscale = np.sum(p["m"] * np.sqrt(p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2))
    for k in ("Px", "Py", "Pz"):
        assert abs(d1[k] - d0[k]) < 1e-14 * pscale
    assert abs(d1["E"] / d0["E"] - 1) < 1e-6


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
def test_circular_orbit_in_halo(orc, scheme):
    # v_c^2 = G M(<r) / r: a particle started on the circle stays on it; the
    # radius error over a quarter turn falls 16x when the step halves
    v2, rc, r0 = 1.0, 1.0, 1.5
    s_ = r0 / rc
    vc = math.sqrt(v2 * (1 - math.atan(s_) / s_))
    T = 2 * math.pi * r0 / vc
    errs = []
    for count in (100, 200):
        p = {"x": [r0], "y": [0.0], "z": [0.0], "vx": [0.0], "vy": [vc], "vz": [0.0], "m": [1.0]}
        s = orc.State(p, halo=orc.Halo(v2, rc))
        getattr(s, "step_" + scheme)(0.25 * T / count, count)
        errs.append(math.hypot(s["x"][0], s["y"][0] - r0))  # ends at (0, r0)
    assert 3.5 < math.log2(errs[0] / errs[1]) < 4.5, errs
    assert errs[1] < 1e-7


def test_force_evaluations_per_step(orc):
    p = wl.plummer(64, 23)
    s = orc.State(p, eps=0.01)
    s.init_jerk()
    orc.reset_force_evals()
    s.step_hermite(1e-3, 5)
    assert orc.force_evals() == 5
    orc.reset_force_evals()
    s.step_rk4(1e-3, 3)
    assert orc.force_evals() == 12


def test_free_particle_exact(orc):
    ic = {"x": [1.0], "y": [2.0], "z": [3.0], "vx": [0.5], "vy": [-0.25], "vz": [0.125], "m": [1.0]}
    for scheme in ("hermite", "rk4"):
        s = orc.State(ic, eps=0.1)
        getattr(s, "step_" + scheme)(0.125, 64)
        assert s["x"][0] == 5.0 and s["y"][0] == 0.0 and s["vz"][0] == 0.125


def test_scales_bound_the_sums(orc):
    # the magnitude sums bound the sums themselves (triangle inequality) and
    # the acceleration scale equals the accel oracle's
    p = wl.plummer(400, 24)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(p, 1.0, 0.01, want_scale=True)
    assert np.all(np.sqrt(ax ** 2 + ay ** 2 + az ** 2) <= A * (1 + 1e-12))
    assert np.all(np.sqrt(jx ** 2 + jy ** 2 + jz ** 2) <= J * (1 + 1e-12))
    A2 = orc.accel(p["x"], p["y"], p["z"], p["m"], 1.0, 0.01, want_scale=True)[3]
    assert np.max(np.abs(A - A2) / A2) < 1e-13


def test_rows_subset_equals_full(orc):
    p = wl.plummer(500, 25)
    halo = orc.Halo(1.0, 1.0)
    full = orc.accel_jerk(p, 1.0, 0.01, halo, want_scale=True)
    rows = np.array([0, 7, 499, 250, 3])
    sub = orc.accel_jerk(p, 1.0, 0.01, halo, want_scale=True, rows=rows)
    for f, g in zip(full, sub):
        assert np.array_equal(f[rows], g)
