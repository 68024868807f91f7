"""Pins for the oracle's softened direct sum, Eqs. (1)-(2) (Section 1).

Each test checks the oracle against something it does not itself compute:
hand-computed values, classical closed forms, exact symmetries of IEEE
arithmetic, scaling laws, a finite-difference gradient of the potential and
an independent extended-precision brute force on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _acc(orc, s, G=1.0, eps=0.0, **kw):
    return orc.accel(s["x"], s["y"], s["z"], s["m"], G, eps, **kw)


def test_two_body_hand_values(orc):
    g = json.load(open(os.path.join(GOLD, "two_body_345.json")))
    ax, ay, az, phi, A = orc.accel(g["x"], g["y"], g["z"], g["m"], g["G"], g["eps"],
                                   want_phi=True, want_scale=True)
    for got, key in ((ax, "ax"), (ay, "ay"), (az, "az"), (phi, "phi"), (A, "A")):
        np.testing.assert_allclose(got, g[key], rtol=1e-15, atol=0, err_msg=key)


def test_two_body_translated_and_rotated_axes(orc):
    # the same 3-4-5 geometry along each axis permutation: catches a
    # transposed or dropped coordinate
    g = json.load(open(os.path.join(GOLD, "two_body_345.json")))
    d = np.array([1.0, 2.0, 2.0])
    for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        dv = d[list(perm)]
        x = np.array([10.0, 10.0 + dv[0]])
        y = np.array([-20.0, -20.0 + dv[1]])
        z = np.array([30.0, 30.0 + dv[2]])
        ax, ay, az = orc.accel(x, y, z, g["m"], 1.0, 4.0)
        got = np.stack([ax, ay, az], 1)
        want = np.array([0.5 * dv / 125.0, -0.25 * dv / 125.0])
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-18)


def _ring(n, R=1.0, tilt=0.3):
    th = 2 * np.pi * np.arange(n) / n
    # ring in a tilted plane so that all three components are exercised
    u = np.array([1.0, 0.0, 0.0])
    v = np.array([0.0, math.cos(tilt), math.sin(tilt)])
    pos = R * (np.cos(th)[:, None] * u + np.sin(th)[:, None] * v)
    return pos


def test_ring_closed_form(orc):
    # N equal masses on a circle, no softening: each feels an inward pull
    # G m / (4 R^2) * sum_{k=1}^{N-1} 1 / sin(pi k / N), potential
    # -G m / (2R) * sum 1 / sin(pi k / N)
    for n in (3, 7, 64):
        R, m, G = 1.7, 0.3, 1.3
        pos = _ring(n, R)
        ks = np.arange(1, n)
        ssum = np.sum(1.0 / np.sin(np.pi * ks / n))
        ax, ay, az, phi = orc.accel(pos[:, 0], pos[:, 1], pos[:, 2], np.full(n, m), G, 0.0,
                                    want_phi=True)
        a = np.stack([ax, ay, az], 1)
        want = -(G * m / (4 * R * R)) * ssum * pos / R
        np.testing.assert_allclose(a, want, rtol=0, atol=2e-14 * n * np.abs(want).max())
        np.testing.assert_allclose(phi, -G * m / (2 * R) * ssum, rtol=1e-13)


def test_cube_softened_closed_form(orc):
    # 8 equal masses at (+-1,+-1,+-1), softening 1: by symmetry each
    # acceleration points to the centre with magnitude
    # G m [3 (2/sqrt3)/5^1.5 + 3 (4/sqrt3)/9^1.5 + (6/sqrt3)/13^1.5]
    c = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    G, m = 2.0, 0.125
    ax, ay, az = orc.accel(c[:, 0], c[:, 1], c[:, 2], np.full(8, m), G, 1.0)
    s3 = math.sqrt(3.0)
    mag = G * m * (3 * (2 / s3) / 5 ** 1.5 + 3 * (4 / s3) / 9 ** 1.5 + (6 / s3) / 13 ** 1.5)
    want = -mag * c / s3
    np.testing.assert_allclose(np.stack([ax, ay, az], 1), want, rtol=1e-14)


def test_pair_antisymmetry_bitwise(orc):
    # IEEE subtraction is sign-symmetric, so for equal masses the two
    # accelerations of a pair are exact negatives of each other
    st = wl.Stream(11)
    for _ in range(20):
        p = st.uniform(6) * 4 - 2
        ax, ay, az = orc.accel(p[0:2], p[2:4], p[4:6], [0.7, 0.7], 1.0, 0.05)
        assert ax[0] == -ax[1] and ay[0] == -ay[1] and az[0] == -az[1]


def test_momentum_balance(orc):
    # Newton's third law: sum_i m_i a_i = 0 up to round-off of the force scale
    st = wl.Stream(5)
    n = 300
    x, y, z = st.normal(n), st.normal(n), st.normal(n)
    m = st.uniform(n)
    ax, ay, az, A = orc.accel(x, y, z, m, 1.0, 0.01, want_scale=True)
    scale = np.sum(m * A)
    for c in (ax, ay, az):
        assert abs(np.sum(m * c)) <= 1e-13 * scale


def test_scaling_laws_exact(orc):
    p = wl.plummer(200, 3)
    ax, ay, az = _acc(orc, p, 1.0, 0.05)
    # (r, eps) -> 2 (r, eps): power-of-two scaling is exact, a -> a / 4
    q = {k: 2.0 * p[k] for k in ("x", "y", "z")}
    q["m"] = p["m"]
    bx, by, bz = _acc(orc, q, 1.0, 0.1)
    assert np.array_equal(bx, ax / 4) and np.array_equal(by, ay / 4) and np.array_equal(bz, az / 4)
    # G -> 2G is exact
    cx, cy, cz = _acc(orc, p, 2.0, 0.05)
    assert np.array_equal(cx, 2 * ax) and np.array_equal(cz, 2 * az)
    # m -> 3m scales linearly (to rounding)
    q = dict(p)
    q["m"] = 3.0 * p["m"]
    dx_, dy_, dz_ = _acc(orc, q, 1.0, 0.05)
    np.testing.assert_allclose(dx_, 3 * ax, rtol=1e-14, atol=1e-14 * np.abs(ax).max())


def test_translation_and_permutation(orc):
    p = wl.plummer(300, 4)
    ax, ay, az, A = _acc(orc, p, 1.0, 0.02, want_scale=True)
    q = dict(p)
    for k, sh in (("x", 1000.0), ("y", -500.0), ("z", 250.0)):
        q[k] = p[k] + sh
    bx, by, bz = _acc(orc, q, 1.0, 0.02)
    # a shift by 1e3 costs about 10 bits of the positions
    assert np.max(np.abs(bx - ax) / A) < 1e-10 and np.max(np.abs(bz - az) / A) < 1e-10
    perm = wl.Stream(9).u64(300).argsort()
    r = {k: p[k][perm] for k in ("x", "y", "z", "m")}
    cx, cy, cz = _acc(orc, r, 1.0, 0.02)
    np.testing.assert_allclose(cx, ax[perm], rtol=0, atol=1e-14 * A.max())
    np.testing.assert_allclose(cy, ay[perm], rtol=0, atol=1e-14 * A.max())


def test_potential_gradient(orc):
    # a_i = -d phi_i / d r_i : central difference of the oracle's own
    # potential, which catches a sign or power mismatch between the two
    p = wl.plummer(64, 6)
    G, eps, h = 1.0, 0.05, 1e-5
    ax, ay, az = _acc(orc, p, G, eps)
    for i in (0, 17, 63):
        for key, comp in (("x", ax), ("y", ay), ("z", az)):
            q = {k: p[k].copy() for k in ("x", "y", "z", "m")}
            q[key][i] += h
            _, _, _, pp = _acc(orc, q, G, eps, want_phi=True)
            q[key][i] -= 2 * h
            _, _, _, pm = _acc(orc, q, G, eps, want_phi=True)
            grad = (pp[i] - pm[i]) / (2 * h)
            assert abs(-grad - comp[i]) < 1e-7 * (abs(comp[i]) + 1e-3)


def test_brute_force_longdouble(orc):
    # independent vectorised brute force in extended precision (80-bit)
    st = wl.Stream(21)
    n = 9
    pos = (st.uniform(3 * n).reshape(3, n) * 2 - 1).astype(np.longdouble)
    m = st.uniform(n).astype(np.longdouble)
    G, eps = np.longdouble(1.5), np.longdouble(0.1)
    d = pos[:, None, :] - pos[:, :, None]           # d[:, i, j] = r_j - r_i
    r2 = (d * d).sum(0) + eps * eps
    w = G * m[None, :] / (r2 * np.sqrt(r2))
    np.fill_diagonal(w, 0)
    want = (w[None] * d).sum(2)
    got = np.stack(orc.accel(*[pos[k].astype(np.float64) for k in range(3)],
                             m.astype(np.float64), 1.5, 0.1), 0)
    np.testing.assert_allclose(got, want.astype(np.float64), rtol=2e-15, atol=1e-16)


def test_plummer_mean_field(orc):
    # mean radial acceleration of a Plummer sphere: -G M r / (r^2 + a^2)^{3/2}
    n = 4096
    p = wl.plummer(n, 1)
    ax, ay, az = _acc(orc, p, 1.0, 0.01)
    r = np.sqrt(p["x"] ** 2 + p["y"] ** 2 + p["z"] ** 2)
    ar = (ax * p["x"] + ay * p["y"] + az * p["z"]) / r
    order = np.argsort(r)
    for b in np.array_split(order[: int(0.95 * n)], 8):
        want = -r[b] / (r[b] ** 2 + 1.0) ** 1.5
        assert abs(np.mean(ar[b]) / np.mean(want) - 1) < 0.08


def test_edge_cases(orc):
    ax, ay, az = orc.accel([], [], [], [], 1.0, 0.1)
    assert ax.size == 0
    ax, ay, az, phi = orc.accel([1.0], [2.0], [3.0], [5.0], 1.0, 0.1, want_phi=True)
    assert ax[0] == 0 and ay[0] == 0 and az[0] == 0 and phi[0] == 0
    # no softening and two coincident particles: their mutual term is zero
    ax, ay, az = orc.accel([0.0, 0.0, 3.0], [0, 0, 4.0], [0, 0, 0], [1.0, 1.0, 2.0], 1.0, 0.0)
    np.testing.assert_allclose(ax[:2], 2.0 * 3.0 / 125.0, rtol=1e-15)
    np.testing.assert_allclose(ay[:2], 2.0 * 4.0 / 125.0, rtol=1e-15)
    assert np.all(np.isfinite(ax))


def test_rows_and_reverse(orc):
    p = wl.plummer(500, 8)
    ax, ay, az, A = _acc(orc, p, 1.0, 0.01, want_scale=True)
    rows = np.array([0, 7, 499, 250])
    bx, by, bz = _acc(orc, p, 1.0, 0.01, rows=rows)
    assert np.array_equal(bx, ax[rows]) and np.array_equal(bz, az[rows])
    cx, cy, cz = _acc(orc, p, 1.0, 0.01, reverse_j=True)
    assert np.max(np.abs(cx - ax) / A) < 1e-13
    # the result does not depend on the thread count
    dx_, _, _ = _acc(orc, p, 1.0, 0.01, nthreads=1)
    ex_, _, _ = _acc(orc, p, 1.0, 0.01, nthreads=3)
    assert np.array_equal(dx_, ex_) and np.array_equal(dx_, ax)
