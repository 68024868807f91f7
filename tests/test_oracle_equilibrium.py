"""Pins of the disk-equilibrium reference (oracle/equilibrium.py), Section 1,
Eqs. (3)-(4), by results fixed independently of its code:
  * Eq. (4) with rho_* = 0 is the self-gravitating isothermal sheet, whose
    solution is rho0 sech^2(z / z0), z0^2 = c_z^2 / (2 pi G rho0), with
    surface density 2 rho0 z0 (Spitzer 1942);
  * with rho_* != 0 the first integral of (ln rho)'' = -k (rho - rho_*),
    (ln rho)'^2 / 2 + k [(rho - rho0) - rho_* ln(rho / rho0)] = 0
    (k = 4 pi G / c_z^2), holds along the solution, and the sign of rho_*
    decides whether the layer is thinner or thicker than the sheet;
  * Eq. (3) gives V_c^2 as the dispersions vanish, and for a flat rotation
    curve, an exponential disk (scale length h) with c_r^2 proportional to
    exp(-R / h) and c_phi^2 = c_r^2 / 2 (the epicyclic ratio of a flat curve)
    it is the closed form V_c^2 + c_r^2 (1/2 - 2 R / h).
NBODY_EQUILIBRIUM_SRC selects another copy of the module (the planted-mistake
tests load mutated copies through it)."""
import importlib.util
import math
import os

import pytest


def _eq():
    alt = os.environ.get("NBODY_EQUILIBRIUM_SRC")
    if not alt:
        from oracle import equilibrium
        return equilibrium
    spec = importlib.util.spec_from_file_location("_equilibrium_under_test", alt)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("rho0,cz2,G", [(2.0, 0.3, 1.0), (0.05, 0.01, 1.0), (7.0, 2.0, 0.5)])
def test_isothermal_sheet(rho0, cz2, G):
    eq = _eq()
    z0 = math.sqrt(cz2 / (2.0 * math.pi * G * rho0))
    zs, rs = eq.vertical_profile(rho0, cz2, 0.0, G, zmax=8.0 * z0, h=z0 / 2000.0)
    assert zs[-1] >= 7.9 * z0  # no early end: the sheet falls all the way
    for z, r in zip(zs[::97], rs[::97]):
        want = rho0 / math.cosh(z / z0) ** 2
        assert abs(r - want) <= 1e-9 * rho0, (z, r, want)
    sigma = eq.column(rho0, cz2, 0.0, G, zmax=30.0 * z0, h=z0 / 2000.0)
    assert abs(sigma - 2.0 * rho0 * z0) <= 1e-8 * sigma


def test_midplane_density_of_the_sheet():
    eq = _eq()
    sigma, cz2, G = 0.4, 0.05, 1.0
    z0_guess = cz2 / (math.pi * G * sigma)   # the sheet's scale height for this column
    rho0 = eq.solve_rho0(sigma, cz2, 0.0, G, zmax=40.0 * z0_guess, h=z0_guess / 1000.0)
    want = math.pi * G * sigma ** 2 / (2.0 * cz2)
    assert abs(rho0 - want) <= 1e-6 * want, (rho0, want)


@pytest.mark.parametrize("frac", [-0.4, -0.1, 0.1, 0.3])
def test_first_integral_with_background(frac):
    eq = _eq()
    rho0, cz2, G = 1.0, 0.2, 1.0
    rs_ = frac * rho0
    k = 4.0 * math.pi * G / cz2
    h = 2e-5
    zs, rs = eq.vertical_profile(rho0, cz2, rs_, G, zmax=0.5, h=h)
    worst = 0.0
    for i in range(1, len(zs) - 1, 50):
        du = (math.log(rs[i + 1]) - math.log(rs[i - 1])) / (2.0 * h)
        inv = 0.5 * du * du + k * ((rs[i] - rho0) - rs_ * math.log(rs[i] / rho0))
        worst = max(worst, abs(inv) / (k * rho0))
    assert worst <= 1e-7, worst
    # a positive rho_* (rising rotation curve) thins the layer, a negative one thickens it
    z0 = math.sqrt(cz2 / (2.0 * math.pi * G * rho0))
    zq, rq = eq.vertical_profile(rho0, cz2, 0.0, G, zmax=0.5, h=h)
    i = int(round(z0 / h))
    sheet = rq[i]
    if frac > 0:
        assert rs[i] > sheet  # (ln rho)'' less negative: slower fall
    else:
        assert rs[i] < sheet


def test_rotation_speed_limits():
    eq = _eq()
    hscale = 1.0
    r = [0.5 + 0.01 * k for k in range(300)]
    vc2 = [1.0] * len(r)
    rho = [math.exp(-x / hscale) for x in r]
    # vanishing dispersions: the circular speed
    tiny = [1e-30 * math.exp(-x / hscale) for x in r]
    v2 = eq.rotation_speed2(r, vc2, rho, tiny, [t / 2.0 for t in tiny])
    assert all(abs(a - 1.0) <= 1e-25 for a in v2)
    # flat curve, exponential disk, c_r^2 ~ exp(-R/h), c_phi^2 = c_r^2 / 2
    c0 = 0.3
    cr2 = [c0 * c0 * math.exp(-x / hscale) for x in r]
    v2 = eq.rotation_speed2(r, vc2, rho, cr2, [c / 2.0 for c in cr2])
    for k in range(1, len(r) - 1):
        want = 1.0 + cr2[k] * (0.5 - 2.0 * r[k] / hscale)
        # central differences on the grid: error O((d ln r)^2), about 1e-4 of c_r^2 here
        assert abs(v2[k] - want) <= 1e-3 * cr2[k], (r[k], v2[k], want)
