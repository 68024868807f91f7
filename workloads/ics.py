"""Seeded synthetic initial conditions for the direct-sum N-body workloads.

These generators produce the input bytes that both the CPU oracle and the GPU
library consume.  They are input recipes only: none of the force sum, the
integrators or the conserved-quantity formulas live here.

Workloads (all in G = 1 units, equal particle masses m = M/N):

* ``plummer``   -- Plummer sphere (Aarseth, Henon & Wielen 1974 sampling),
  scale a, total mass M, untruncated, moved to the centre-of-mass frame.
* ``exp_disk``  -- the gravitationally unstable exponential stellar disk used
  for the paper's galactic-disk runs (Section 3): surface density
  ~ exp(-R/h) cut at R = 4h, vertical sech^2(z/z0), rotation set by the
  enclosed mass of disk plus a fixed cored isothermal halo (or of the disk
  alone with ``halo=no_halo()``, the paper's self-gravitating case), radial dispersion
  from a Toomre Q, azimuthal dispersion from the epicyclic ratio and mean
  rotation from the radial Jeans (asymmetric-drift) balance of Eq. (3).
  The paper builds its disks with an iterative equilibrium method that it
  does not spell out; this is a simpler stand-in with the same structure.
* ``kepler_pair`` -- two bodies on a bound Kepler orbit, started at pericentre.
* ``batch_mix`` -- many independent systems of uneven N packed back to back.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .rng import Stream

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m")


@dataclass
class HaloSpec:
    """Cored (pseudo-)isothermal sphere rho = rho0 / (1 + r^2/rc^2).

    v2 is the asymptotic circular speed squared, V_inf^2 = 4 pi G rho0 rc^2.
    """

    v2: float
    rc: float


def default_halo(h: float = 1.0, md: float = 1.0, G: float = 1.0) -> HaloSpec:
    """Halo with core radius h holding the disk's mass inside 4h.

    The enclosed mass of the cored sphere is (v2/G) (r - rc atan(r/rc)), so
    requiring M_h(<4h) = M_d gives v2 = G M_d / (4h - h atan 4).
    """
    rc = h
    v2 = G * md / (4.0 * h - rc * math.atan(4.0 * h / rc))
    return HaloSpec(v2=v2, rc=rc)


def no_halo() -> HaloSpec:
    """No external field: the completely self-gravitating disk of the paper's
    Section 2, whose rotation comes from the disk's own enclosed mass."""
    return HaloSpec(v2=0.0, rc=1.0)


def outer_period(h: float = 1.0, rmax_h: float = 4.0, md: float = 1.0, halo: HaloSpec | None = None,
                 G: float = 1.0) -> float:
    """Rotation period 2 pi R / v_c(R) at the disk's edge R = rmax_h h, with
    v_c^2 = G M(<R) / R as in exp_disk (the disk's whole mass is inside)."""
    halo = default_halo(h, md, G) if halo is None else halo
    R = rmax_h * h
    m = md + (halo.v2 / G) * (R - halo.rc * math.atan(R / halo.rc))
    return 2.0 * math.pi * R / math.sqrt(G * m / R)


def _com_frame(d: dict) -> dict:
    m = d["m"]
    M = m.sum()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        d[k] = d[k] - (m * d[k]).sum() / M
    return d


def plummer(n: int, seed: int, a: float = 1.0, M: float = 1.0, G: float = 1.0) -> dict:
    """Plummer sphere sampled from its distribution function.

    Radius from the inverted cumulative mass r = a (u^{-2/3} - 1)^{-1/2};
    speed q v_esc(r) with v_esc = sqrt(2GM/a) (1 + r^2/a^2)^{-1/4} and q drawn
    by rejection from g(q) = q^2 (1 - q^2)^{7/2}; isotropic directions.
    """
    s = Stream(seed)
    out = {k: np.zeros(n) for k in FIELDS}
    if n == 0:
        return out
    u = s.uniform(n)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    ct = 2.0 * s.uniform(n) - 1.0
    ph = 2.0 * np.pi * s.uniform(n)
    st = np.sqrt(1.0 - ct * ct)
    out["x"] = r * st * np.cos(ph)
    out["y"] = r * st * np.sin(ph)
    out["z"] = r * ct
    # rejection sampling of q, vectorised in rounds
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        k = todo.size
        x1 = s.uniform(2 * k + 16)
        x2 = 0.1 * s.uniform(2 * k + 16)
        ok = x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        acc = x1[ok][:k]
        q[todo[: acc.size]] = acc
        todo = todo[acc.size:]
    ve = math.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    v = q * ve
    ct = 2.0 * s.uniform(n) - 1.0
    ph = 2.0 * np.pi * s.uniform(n)
    st = np.sqrt(1.0 - ct * ct)
    out["vx"] = v * st * np.cos(ph)
    out["vy"] = v * st * np.sin(ph)
    out["vz"] = v * ct
    out["m"] = np.full(n, M / n)
    return _com_frame(out)


def _disk_mass_fraction(R: np.ndarray, h: float, rmax_h: float) -> np.ndarray:
    t = R / h
    return (1.0 - (1.0 + t) * np.exp(-t)) / (1.0 - (1.0 + rmax_h) * math.exp(-rmax_h))


def exp_disk(
    n: int,
    seed: int,
    h: float = 1.0,
    rmax_h: float = 4.0,
    z0: float = 0.1,
    md: float = 1.0,
    Q: float = 1.2,
    halo: HaloSpec | None = None,
    G: float = 1.0,
) -> dict:
    """Exponential disk with a fixed cored-isothermal halo (see module doc)."""
    if halo is None:
        halo = default_halo(h, md, G)
    s = Stream(seed)
    out = {k: np.zeros(n) for k in FIELDS}
    if n == 0:
        return out
    rmax = rmax_h * h
    # radius by bisection on the truncated enclosed-mass fraction
    u = s.uniform(n)
    lo = np.zeros(n)
    hi = np.full(n, rmax)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = _disk_mass_fraction(mid, h, rmax_h) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    R = 0.5 * (lo + hi)
    phi = 2.0 * np.pi * s.uniform(n)
    zz = z0 * np.arctanh(2.0 * s.uniform(n) - 1.0)

    norm = md / (2.0 * np.pi * h * h * (1.0 - (1.0 + rmax_h) * math.exp(-rmax_h)))

    def sigma(Rv):
        return norm * np.exp(-Rv / h)

    def m_enc(Rv):
        md_in = md * _disk_mass_fraction(np.minimum(Rv, rmax), h, rmax_h)
        mh_in = (halo.v2 / G) * (Rv - halo.rc * np.arctan(Rv / halo.rc))
        return md_in + mh_in

    def dm_dR(Rv):
        rho_h = halo.v2 / (4.0 * np.pi * G * halo.rc ** 2) / (1.0 + (Rv / halo.rc) ** 2)
        return 2.0 * np.pi * Rv * sigma(Rv) + 4.0 * np.pi * Rv * Rv * rho_h

    Rs = np.maximum(R, 1e-6 * h)
    M_in = m_enc(Rs)
    vc2 = G * M_in / Rs
    om2 = G * M_in / Rs ** 3
    kap2 = om2 + G * dm_dR(Rs) / Rs ** 2
    kap = np.sqrt(kap2)

    def sig_r(Rv):
        Mv = m_enc(Rv)
        k2 = G * Mv / Rv ** 3 + G * dm_dR(Rv) / Rv ** 2
        return 3.36 * Q * G * sigma(Rv) / np.sqrt(k2)

    sR = sig_r(Rs)
    sphi2 = sR ** 2 * kap2 / (4.0 * om2)
    sz = np.sqrt(np.pi * G * sigma(Rs) * z0)
    # d ln(Sigma sigma_R^2) / d ln R by a central difference in ln R
    dl = 1e-4
    Rp, Rm = Rs * math.exp(dl), Rs * math.exp(-dl)
    dlog = (np.log(sigma(Rp) * sig_r(Rp) ** 2) - np.log(sigma(Rm) * sig_r(Rm) ** 2)) / (2 * dl)
    vphi2 = vc2 + sR ** 2 * (1.0 - sphi2 / sR ** 2 + dlog)
    vphi_mean = np.sqrt(np.maximum(vphi2, 0.0))

    vR = sR * s.normal(n)
    vphi = vphi_mean + np.sqrt(sphi2) * s.normal(n)
    vz = sz * s.normal(n)
    c, sn = np.cos(phi), np.sin(phi)
    out["x"] = R * c
    out["y"] = R * sn
    out["z"] = zz
    out["vx"] = vR * c - vphi * sn
    out["vy"] = vR * sn + vphi * c
    out["vz"] = vz
    out["m"] = np.full(n, md / n)
    return _com_frame(out)


def kepler_pair(e: float = 0.5, a: float = 1.0, m1: float = 0.5, m2: float = 0.5, G: float = 1.0) -> dict:
    """Two bodies at pericentre of a Kepler orbit, centre-of-mass frame.

    Relative orbit: r_p = a (1 - e), v_p = sqrt(G M (1 + e) / (a (1 - e))).
    """
    M = m1 + m2
    rp = a * (1.0 - e)
    vp = math.sqrt(G * M * (1.0 + e) / (a * (1.0 - e)))
    out = {k: np.zeros(2) for k in FIELDS}
    out["x"] = np.array([-m2 / M * rp, m1 / M * rp])
    out["vy"] = np.array([-m2 / M * vp, m1 / M * vp])
    out["m"] = np.array([m1, m2])
    return out


def kepler_relative_position(t: float, e: float = 0.5, a: float = 1.0, M: float = 1.0, G: float = 1.0):
    """Exact relative separation (x, y) at time t after pericentre, from
    Kepler's equation M = E - e sin E solved by Newton iteration."""
    n_mean = math.sqrt(G * M / a ** 3)
    Mn = math.fmod(n_mean * t, 2.0 * math.pi)
    E = Mn if e < 0.8 else math.pi
    for _ in range(100):
        dE = (E - e * math.sin(E) - Mn) / (1.0 - e * math.cos(E))
        E -= dE
        if abs(dE) < 1e-16:
            break
    x = a * (math.cos(E) - e)
    y = a * math.sqrt(1.0 - e * e) * math.sin(E)
    return x, y


def batch_sizes(B: int, seed: int, lo_log2: int = 10, hi_log2: int = 16) -> np.ndarray:
    """N_k = round(2^(lo + (hi - lo) u_k)), log-uniform in [2^lo, 2^hi]."""
    u = Stream(seed).uniform(B)
    return np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def batch_mix(B: int = 256, seed: int = 4, lo_log2: int = 10, hi_log2: int = 16, sizes=None) -> dict:
    """B independent systems packed back to back: systems k < B/2 are Plummer
    spheres, the rest exponential disks; system k uses seed 1000 + k.
    Returns the packed SoA arrays plus ``off`` (B + 1 offsets) and ``kind``."""
    if sizes is None:
        sizes = batch_sizes(B, seed, lo_log2, hi_log2)
    parts, kinds = [], []
    for k, nk in enumerate(sizes):
        if k < B // 2:
            parts.append(plummer(int(nk), 1000 + k))
            kinds.append("plummer")
        else:
            parts.append(exp_disk(int(nk), 1000 + k))
            kinds.append("disk")
    out = {f: np.concatenate([p[f] for p in parts]) if parts else np.zeros(0) for f in FIELDS}
    out["off"] = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out["kind"] = kinds
    return out


def request_stream(
    count: int,
    seed: int,
    rate: float,
    lo_log2: int = 12,
    hi_log2: int = 20,
    steps_lo: int = 10,
    steps_hi: int = 1000,
    fp64_fraction: float = 0.1,
) -> list[dict]:
    """Poisson arrivals of integration requests: exponential inter-arrival
    gaps at the given rate, N log-uniform in [2^lo, 2^hi], steps uniform in
    [steps_lo, steps_hi], model Plummer or disk with equal odds, and an FP64
    flag set on a fraction of requests."""
    s = Stream(seed)
    gaps = -np.log(s.uniform(count)) / rate
    t = np.cumsum(gaps)
    n = np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * s.uniform(count))).astype(np.int64)
    steps = steps_lo + np.floor((steps_hi - steps_lo + 1) * s.uniform(count)).astype(np.int64)
    model = np.where(s.uniform(count) < 0.5, "plummer", "disk")
    fp64 = s.uniform(count) < fp64_fraction
    return [
        dict(id=k, t_arrive=float(t[k]), n=int(n[k]), steps=int(steps[k]), model=str(model[k]),
             fp64=bool(fp64[k]), seed=50000 + k)
        for k in range(count)
    ]


def make(kind: str, n: int, seed: int) -> dict:
    if kind == "plummer":
        return plummer(n, seed)
    if kind == "disk":
        return exp_disk(n, seed)
    if kind == "disk_sg":
        return exp_disk(n, seed, halo=no_halo())
    raise ValueError(f"unknown workload {kind!r}")
