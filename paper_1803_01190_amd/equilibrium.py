"""Disk initial conditions in equilibrium, Section 1, Eqs. (3)-(4), built by
iterating with the library's own float64 force sums.

The paper builds its disks with an iterative equilibrium procedure from its
references, which it does not describe beyond the two balance equations.
Here the exponential disk of the workload recipe (surface density
~ exp(-R/h) cut at 4h, sech^2 layers, rotation from the spherical enclosed
mass) is the start, and each iteration
  1. sums the accelerations of all particles on the GPU (nbody_accel,
     float64, plus the halo when there is one);
  2. takes, in radial bins of equal particle count, the circular speed
     V_c^2 = R <-a_R> of the bin (smoothed by a least-squares polynomial in
     R, whose derivative gives kappa^2 = dV_c^2/dR / R + 2 V_c^2 / R^2 and
     rho_* = dV_c^2/dR / (4 pi G R));
  3. solves Eq. (4) in each bin for the layer with the bin's surface density
     and vertical dispersion c_z^2 = pi G Sigma z0 (the isothermal sheet of
     thickness z0 that the recipe starts from), with the bin's rho_* (less
     the halo's midplane density, which the layer also feels), and moves
     every particle to the height of the same quantile in that layer
     (interpolated between neighbouring bins);
  4. sets the velocities from Eq. (3): sigma_R = 3.36 Q G Sigma / kappa
     (Toomre Q), sigma_phi^2 = sigma_R^2 kappa^2 / (4 Omega^2), mean rotation
     v_phi^2 = V_c^2 + sigma_R^2 (1 - sigma_phi^2 / sigma_R^2
     + d ln(rho0 sigma_R^2) / d ln R) (clamped at 0) with rho0 the layer's
     midplane density, and sigma_z = c_z, drawing the same seeded normal
     deviates every iteration; then moves to the centre-of-mass frame.
Radii, azimuths and masses never change, so the surface density keeps the
recipe's profile exactly.

Reading of the paper: Eq. (3) is taken with v_phi^2 / r on its left (the
printed v_phi / r is not dimensionally consistent) and the <v_r v_z> terms
of Eqs. (3)-(4) are dropped (a thin disk with aligned velocity ellipsoid).
"""
from __future__ import annotations

import math

import numpy as np

from . import nbody as nb


def _layer(rho0: np.ndarray, cz2: np.ndarray, rstar: np.ndarray, G: float, z: np.ndarray) -> np.ndarray:
    """Eq. (4) for many bins at once: densities on the height grid z (from
    0, uniform step) by the classical RK4 on u = ln rho, u'' = -k (rho - rho_*),
    each bin's layer ending where its density stops falling (zero beyond)."""
    k4 = 4.0 * math.pi * G / cz2
    h = z[1] - z[0]
    u = np.log(rho0)
    w = np.zeros_like(u)
    out = np.zeros((z.size, rho0.size))
    out[0] = rho0
    live = np.ones(rho0.size, dtype=bool)

    def f(u, w):
        return w, -k4 * (np.exp(u) - rstar)

    for i in range(1, z.size):
        a1, b1 = f(u, w)
        a2, b2 = f(u + 0.5 * h * a1, w + 0.5 * h * b1)
        a3, b3 = f(u + 0.5 * h * a2, w + 0.5 * h * b2)
        a4, b4 = f(u + h * a3, w + h * b3)
        un = u + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
        wn = w + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
        live &= ~((wn >= 0.0) & (i > 1))
        u = np.where(live, un, u)
        w = np.where(live, wn, w)
        out[i] = np.where(live, np.exp(u), 0.0)
    return out


def _columns(prof: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Cumulative 2 * integral of rho from 0 to each height (trapezoids)."""
    h = z[1] - z[0]
    c = np.zeros_like(prof)
    c[1:] = np.cumsum(0.5 * (prof[1:] + prof[:-1]) * h, axis=0)
    return 2.0 * c


def _midplane(sigma: np.ndarray, cz2: np.ndarray, rstar: np.ndarray, G: float, z: np.ndarray) -> np.ndarray:
    """Midplane densities whose layers hold the surface densities sigma
    (bisection in log rho0, all bins together)."""
    lo = np.full(sigma.size, 1e-8)
    hi = np.full(sigma.size, 1e8)
    for _ in range(48):
        mid = np.sqrt(lo * hi)
        col = _columns(_layer(mid, cz2, rstar, G, z), z)[-1]
        lo = np.where(col < sigma, mid, lo)
        hi = np.where(col < sigma, hi, mid)
    return np.sqrt(lo * hi)


def _fit(x: np.ndarray, y: np.ndarray, deg: int):
    """Least-squares polynomial in x / max(x) and its derivative in x."""
    s = float(x.max())
    c = np.polynomial.polynomial.polyfit(x / s, y, deg)
    d = np.polynomial.polynomial.polyder(c) / s
    return (lambda t: np.polynomial.polynomial.polyval(t / s, c)), (lambda t: np.polynomial.polynomial.polyval(t / s, d))


def equilibrium_disk(ctx, ic: dict, *, h: float = 1.0, z0: float = 0.1, Q: float = 1.2, G: float = 1.0,
                     eps: float = 0.02, halo=None, seed: int = 0, iters: int = 3, nbins: int = 48,
                     deg: int = 8, info: dict | None = None) -> dict:
    """Iterate the exponential-disk initial conditions ic (scale length h,
    sech^2 thickness z0) towards the balance of Eqs. (3)-(4) under the
    library's float64 forces (softening eps, optional halo with attributes
    v2 and rc); returns new initial conditions (same radii, azimuths and
    masses).  info, if given, receives per-iteration diagnostics."""
    import torch

    x0, y0 = np.asarray(ic["x"], float), np.asarray(ic["y"], float)
    z = np.asarray(ic["z"], float).copy()
    m = np.asarray(ic["m"], float)
    n = x0.size
    R = np.hypot(x0, y0)
    cph, sph = x0 / np.maximum(R, 1e-300), y0 / np.maximum(R, 1e-300)
    M = float(m.sum())
    rmax = 4.0 * h
    norm = M / (2.0 * math.pi * h * h * (1.0 - 5.0 * math.exp(-4.0)))
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((3, n))
    # the quantile of each particle in its layer (the recipe's sech^2 layers)
    qz = 0.5 * (1.0 + np.tanh(z / z0))
    # radial bins of equal particle count
    edges = np.quantile(R, np.linspace(0.0, 1.0, nbins + 1))
    edges[0], edges[-1] = 0.0, max(edges[-1], rmax)
    rc = 0.5 * (edges[1:] + edges[:-1])
    which = np.clip(np.searchsorted(edges, R, side="right") - 1, 0, nbins - 1)
    sig_b = norm * np.exp(-rc / h)
    cz2_b = math.pi * G * sig_b * z0
    zgrid = np.linspace(0.0, 12.0 * z0, 2401)
    prm = nb.Params(G=G, eps=eps, prec=nb.NB_FP64, halo=halo is not None,
                    halo_v2=halo.v2 if halo is not None else 0.0, halo_rc=halo.rc if halo is not None else 0.0)
    vel = None
    for it in range(iters):
        cur = {"x": x0, "y": y0, "z": z, "m": m, "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n)}
        s = nb.System.from_arrays(cur)
        nb.nbody_accel(ctx, s, prm)
        torch.cuda.synchronize()
        ax, ay = s["ax"].cpu().numpy(), s["ay"].cpu().numpy()
        del s
        # 2. rotation curve from the particles' own forces
        ar = ax * cph + ay * sph
        vc2_b = np.bincount(which, weights=-R * ar * m, minlength=nbins) / np.bincount(which, weights=m, minlength=nbins)
        vc2f, dvc2f = _fit(rc, vc2_b, deg)
        vc2, dvc2 = np.maximum(vc2f(rc), 1e-12), dvc2f(rc)
        kap2 = np.maximum(dvc2 / rc + 2.0 * vc2 / rc ** 2, 1e-12)
        om2 = vc2 / rc ** 2
        rstar = dvc2 / (4.0 * math.pi * G * rc)
        if halo is not None:
            # the halo's density at the bin's radius in the midplane
            rstar = rstar - halo.v2 / (4.0 * math.pi * G * (halo.rc ** 2 + rc ** 2))
        # 3. vertical balance: layers of each bin, particles at their quantiles
        rho0 = _midplane(sig_b, cz2_b, rstar, G, zgrid)
        prof = _layer(rho0, cz2_b, rstar, G, zgrid)
        cum = _columns(prof, zgrid) / sig_b          # fraction of the column within |z|
        frac = np.abs(2.0 * qz - 1.0)                # fraction within the particle's |z|
        zn = np.empty(n)
        for b in range(nbins):
            sel = which == b
            zn[sel] = np.interp(frac[sel], cum[:, b], zgrid)
        z = np.sign(qz - 0.5) * zn
        # 4. radial balance, Eq. (3)
        sr2 = (3.36 * Q * G * sig_b) ** 2 / kap2
        sp2 = sr2 * kap2 / (4.0 * om2)
        lr = np.log(rho0 * sr2)
        dlog = np.gradient(lr, np.log(rc))
        vphi2 = np.maximum(vc2 + sr2 * (1.0 - sp2 / sr2 + dlog), 0.0)
        # particle values interpolated in R between bin centres
        vphi = np.sqrt(np.interp(R, rc, vphi2))
        sR, sP = np.sqrt(np.interp(R, rc, sr2)), np.sqrt(np.interp(R, rc, sp2))
        sZ = np.sqrt(np.interp(R, rc, cz2_b))
        vr, vp, vz = sR * g[0], vphi + sP * g[1], sZ * g[2]
        vel = (vr * cph - vp * sph, vr * sph + vp * cph, vz)
        if info is not None:
            info.setdefault("vc2", []).append(vc2.tolist())
            info.setdefault("rho0", []).append(rho0.tolist())
    out = {"x": x0.copy(), "y": y0.copy(), "z": z, "m": m.copy(), "vx": vel[0], "vy": vel[1], "vz": vel[2]}
    # centre-of-mass frame
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        out[k] = out[k] - float((m * out[k]).sum()) / M
    out["ax"], out["ay"], out["az"] = np.zeros(n), np.zeros(n), np.zeros(n)
    if info is not None:
        info["bins"] = rc.tolist()
    return out
