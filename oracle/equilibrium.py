"""Equilibrium of a collisionless stellar disk, Section 1, Eqs. (3)-(4) --
TEST INFRASTRUCTURE (the plain reference that the library's iterated disk
initial conditions are checked against; only tests may use it).  Plain
loops, float64, no vectorised numerics.

Eq. (4), the vertical balance of a thin layer whose vertical dispersion c_z
does not depend on z, with the <v_r v_z> term dropped:
    rho rho'' - rho'^2 + (4 pi G rho^2 / c_z^2) (rho - rho_*) = 0,
    rho_* = (1 / (4 pi G r)) dV_c^2 / dr.
Dividing by rho^2 it reads (ln rho)'' = -(4 pi G / c_z^2) (rho - rho_*); it is
integrated from the midplane, ln rho(0) = ln rho0 and (ln rho)'(0) = 0, by
the classical fourth-order Runge-Kutta method with a fixed step, up to the
first height where the density stops falling (when rho_* > 0 the layer ends
at its minimum) or zmax.

Eq. (3), the radial balance, read with v_phi^2 / r on the left (as printed it
has v_phi / r, which is not dimensionally consistent) and the <v_r v_z> term
dropped:
    v_phi^2 = V_c^2 + c_r^2 (1 - c_phi^2 / c_r^2 + d ln(rho c_r^2) / d ln r),
with V_c^2 = r dPsi/dr the circular speed (the sign of the printed dPsi/dr
term depends on the potential's sign convention; the gravitational pull
gives the circular speed).  The logarithmic derivative is taken by central
differences on the caller's radial grid (one-sided at its ends).
"""
from __future__ import annotations

import math


def vertical_profile(rho0: float, cz2: float, rho_star: float = 0.0, G: float = 1.0, zmax: float = 2.0,
                     h: float = 1e-4):
    """Heights z_k = k h and densities rho(z_k) of Eq. (4) from the
    midplane up; returns (z, rho) as lists."""
    k4 = 4.0 * math.pi * G / cz2

    def f(u, w):  # u = ln rho, w = u'
        return w, -k4 * (math.exp(u) - rho_star)

    u, w = math.log(rho0), 0.0
    zs, rs = [0.0], [rho0]
    z = 0.0
    while z < zmax:
        a1, b1 = f(u, w)
        a2, b2 = f(u + 0.5 * h * a1, w + 0.5 * h * b1)
        a3, b3 = f(u + 0.5 * h * a2, w + 0.5 * h * b2)
        a4, b4 = f(u + h * a3, w + h * b3)
        u_new = u + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
        w_new = w + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
        if w_new >= 0.0 and z > 0.0:
            break  # the density has stopped falling: end of the layer
        u, w = u_new, w_new
        z += h
        zs.append(z)
        rs.append(math.exp(u))
    return zs, rs


def column(rho0: float, cz2: float, rho_star: float = 0.0, G: float = 1.0, zmax: float = 2.0,
           h: float = 1e-4) -> float:
    """Surface density 2 * integral of rho over z >= 0 (trapezoid rule)."""
    zs, rs = vertical_profile(rho0, cz2, rho_star, G, zmax, h)
    s = 0.0
    for k in range(1, len(zs)):
        s += 0.5 * (rs[k] + rs[k - 1]) * (zs[k] - zs[k - 1])
    return 2.0 * s


def solve_rho0(sigma: float, cz2: float, rho_star: float = 0.0, G: float = 1.0, zmax: float = 2.0,
               h: float = 1e-4, iters: int = 60) -> float:
    """Midplane density whose layer has surface density sigma (bisection in
    log rho0; the column grows with rho0)."""
    lo, hi = 1e-12, 1e12
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if column(mid, cz2, rho_star, G, zmax, h) < sigma:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def rotation_speed2(r, vc2, rho, cr2, cphi2):
    """Eq. (3) on a radial grid r (increasing): mean azimuthal speed squared
    from the circular speed squared vc2, the midplane density rho and the
    dispersions squared cr2, cphi2 (lists of equal length)."""
    n = len(r)
    out = []
    for k in range(n):
        a, b = (k - 1, k + 1) if 0 < k < n - 1 else ((k, k + 1) if k == 0 else (k - 1, k))
        dlog = (math.log(rho[b] * cr2[b]) - math.log(rho[a] * cr2[a])) / (math.log(r[b]) - math.log(r[a]))
        out.append(vc2[k] + cr2[k] * (1.0 - cphi2[k] / cr2[k] + dlog))
    return out
