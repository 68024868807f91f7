"""Pins for the oracle's fixed external halo (cored isothermal sphere).

The paper's disk is fully self-gravitating (Section 1); the disk workloads
here add a fixed analytic halo, so the oracle carries it as an optional
field.  Pinned by hand-computed values, the asymptotic flat rotation curve,
the potential's derivative and continuity of the small-radius series.
"""
import math

import numpy as np


def _halo(orc, r, v2=0.37, rc=1.3, direction=(0.6, 0.0, 0.8)):
    d = np.asarray(direction)
    x, y, z = (np.atleast_1d(r)[:, None] * d).T
    ax, ay, az, phi = orc.halo_accel(x, y, z, orc.Halo(v2, rc), want_phi=True)
    return np.stack([ax, ay, az], 1), phi


def test_value_at_core_radius(orc):
    # at r = rc: V_c^2 = V_inf^2 (1 - atan(1)) = V_inf^2 (1 - pi/4)
    v2, rc = 0.37, 1.3
    a, phi = _halo(orc, rc, v2, rc)
    mag = np.linalg.norm(a[0])
    assert abs(mag * rc / (v2 * (1 - math.pi / 4)) - 1) < 1e-14
    # Phi(rc) = V_inf^2 (pi/4 + ln(2)/2)
    assert abs(phi[0] / (v2 * (math.pi / 4 + 0.5 * math.log(2.0))) - 1) < 1e-14


def test_points_inward(orc):
    d = np.array([0.6, 0.0, 0.8])
    a, _ = _halo(orc, np.array([0.01, 1.0, 7.0]), direction=d)
    for row in a:
        cos = row @ d / np.linalg.norm(row)
        assert abs(cos + 1) < 1e-15


def test_flat_rotation_curve(orc):
    # r |a| -> V_inf^2 (1 - pi rc / (2 r) + rc^2/r^2) for r >> rc
    v2, rc = 0.37, 1.3
    r = 1e4 * rc
    a, _ = _halo(orc, r, v2, rc)
    vc2 = r * np.linalg.norm(a[0])
    s = r / rc
    assert abs(vc2 / (v2 * (1 - math.pi / (2 * s) + 1 / s ** 2)) - 1) < 1e-11


def test_potential_derivative(orc):
    # d Phi / dr = |a| (= V_c^2 / r)
    v2, rc = 0.37, 1.3
    for r in (1e-3, 0.2, 1.0, 3.0, 40.0):
        # in the harmonic core a wider step keeps the difference above round-off
        h = (0.1 if r < 0.01 else 1e-5) * r
        _, pp = _halo(orc, r + h, v2, rc)
        _, pm = _halo(orc, r - h, v2, rc)
        a, _ = _halo(orc, r, v2, rc)
        fd = (pp[0] - pm[0]) / (2 * h)
        assert abs(fd / np.linalg.norm(a[0]) - 1) < 1e-6, r


def test_series_branch_continuity(orc):
    # the small-radius branch (series below r = rc/2) joins the closed form
    v2, rc = 0.37, 1.3
    r0 = 0.5 * rc
    a_lo, p_lo = _halo(orc, np.nextafter(r0, 0.0), v2, rc)
    a_hi, p_hi = _halo(orc, r0, v2, rc)
    assert abs(np.linalg.norm(a_lo[0]) / np.linalg.norm(a_hi[0]) - 1) < 1e-13
    assert abs(p_lo[0] / p_hi[0] - 1) < 1e-14
    # near the centre the field is harmonic: |a| = V_inf^2 r / (3 rc^2) (1 - 3 s^2/5)
    for s in (1e-9, 1e-5, 1e-3):
        a, _ = _halo(orc, s * rc, v2, rc)
        want = v2 * s / (3 * rc) * (1 - 0.6 * s * s + (3.0 / 7) * s ** 4)
        assert abs(np.linalg.norm(a[0]) / want - 1) < 1e-14
    # at the centre: zero field, Phi(0) = V_inf^2
    a0, p0 = _halo(orc, 0.0, v2, rc)
    assert np.all(a0 == 0) and p0[0] == v2


def test_series_matches_high_precision(orc):
    # 1 - atan(s)/s against an independent extended-precision evaluation
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    v2, rc = 1.0, 1.0

    def atan_dec(s):
        # atan by its Euler series, convergent for all s: atan s = sum
        # 2^{2k} (k!)^2 / (2k+1)! * s^{2k+1} / (1+s^2)^{k+1}
        s = Decimal(s)
        q = s * s / (1 + s * s)
        term = s / (1 + s * s)
        tot = Decimal(0)
        for k in range(400):
            tot += term
            term = term * q * (2 * k + 2) / (2 * k + 3)
        return tot

    for s in (1e-3, 0.05, 0.3, 0.49, 0.51, 2.0):
        a, _ = _halo(orc, s, v2, rc, direction=(1.0, 0.0, 0.0))
        want = float((1 - atan_dec(s) / Decimal(s)) / (Decimal(s) * Decimal(s))) * s
        assert abs(-a[0][0] / want - 1) < 5e-15, s
