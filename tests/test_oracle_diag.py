"""Pins for the oracle's conserved quantities, Eqs. (8)-(10) (Section 3).

Pinned by the Kepler pair's closed forms, the ring's closed-form binding
energy, exact momentum and angular momentum of rigid motions, the external
potential at the halo centre, consistency with the accelerations' potential,
and the Plummer sphere's energy and virial ratio.
"""
import json
import math
import os

import numpy as np

import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_kepler_closed_forms(orc):
    g = json.load(open(os.path.join(GOLD, "kepler_e05.json")))
    d = orc.diag(wl.kepler_pair(), 1.0, 0.0)
    for k in ("E", "W", "K", "Lz"):
        assert abs(d[k] - g[k]) < 1e-15, k
    assert d["M"] == 1.0
    assert abs(d["Px"]) < 1e-16 and abs(d["Py"]) < 1e-16 and d["Lx"] == 0 and d["Ly"] == 0


def test_two_body_hand_potential(orc):
    g = json.load(open(os.path.join(GOLD, "two_body_345.json")))
    s = {k: np.asarray(g[k], float) for k in ("x", "y", "z", "m")}
    for k in ("vx", "vy", "vz"):
        s[k] = np.zeros(2)
    d = orc.diag(s, g["G"], g["eps"])
    assert abs(d["W"] - g["W"]) < 1e-17 and d["K"] == 0


def test_ring_binding_energy(orc):
    # W = -(N/2) G m^2 / (2R) * sum_{k=1}^{N-1} 1/sin(pi k/N)
    n, R, m, G = 12, 2.0, 0.1, 1.0
    th = 2 * np.pi * np.arange(n) / n
    s = {"x": R * np.cos(th), "y": R * np.sin(th), "z": np.zeros(n), "m": np.full(n, m)}
    w = 0.7  # rigid rotation about z: v = w (-y, x, 0)
    s["vx"], s["vy"], s["vz"] = -w * s["y"], w * s["x"], np.zeros(n)
    d = orc.diag(s, G, 0.0)
    ssum = np.sum(1 / np.sin(np.pi * np.arange(1, n) / n))
    assert abs(d["W"] / (-(n / 2) * G * m * m / (2 * R) * ssum) - 1) < 1e-14
    # K = M (w R)^2 / 2, L_z = M R^2 w, P = 0
    assert abs(d["K"] / (n * m * (w * R) ** 2 / 2) - 1) < 1e-14
    assert abs(d["Lz"] / (n * m * R * R * w) - 1) < 1e-14
    assert abs(d["Px"]) < 1e-15 and abs(d["Py"]) < 1e-15


def test_uniform_translation(orc):
    p = wl.plummer(100, 2)
    s = dict(p)
    s["vx"], s["vy"], s["vz"] = np.full(100, 0.5), np.full(100, -2.0), np.full(100, 0.25)
    d = orc.diag(s, 1.0, 0.01)
    M = p["m"].sum()
    assert abs(d["Px"] - 0.5 * M) < 1e-14 and abs(d["Py"] + 2.0 * M) < 1e-14
    assert abs(d["K"] - 0.5 * M * (0.25 + 4 + 0.0625)) < 1e-14
    # centre of mass of a shifted cloud
    s["x"] = p["x"] + 3.0
    d = orc.diag(s, 1.0, 0.01)
    assert abs(d["Cx"] - 3.0) < 1e-14 and abs(d["Cy"]) < 1e-14


def test_halo_potential_energy(orc):
    s = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
    s["m"] = np.array([2.0])
    d = orc.diag(s, 1.0, 0.1, orc.Halo(0.37, 1.3))
    # Phi(0) = V_inf^2
    assert d["Wext"] == 2.0 * 0.37 and d["E"] == d["Wext"]


def test_potential_energy_matches_accel_potential(orc):
    # W = (1/2) sum_i m_i phi_i with phi from the force pass
    p = wl.plummer(400, 3)
    _, _, _, phi = orc.accel(p["x"], p["y"], p["z"], p["m"], 1.0, 0.02, want_phi=True)
    d = orc.diag(p, 1.0, 0.02)
    assert abs(d["W"] / (0.5 * np.sum(p["m"] * phi)) - 1) < 1e-13


def test_brute_force_longdouble(orc):
    st = wl.Stream(31)
    n = 7
    a = (st.uniform(6 * n).reshape(6, n) * 2 - 1).astype(np.longdouble)
    m = st.uniform(n).astype(np.longdouble)
    G, eps = np.longdouble(1.2), np.longdouble(0.05)
    d = a[:3, None, :] - a[:3, :, None]
    r = np.sqrt((d * d).sum(0) + eps * eps)
    pair = G * m[:, None] * m[None, :] / r
    np.fill_diagonal(pair, 0)
    W = -pair.sum() / 2
    K = (m * (a[3:] ** 2).sum(0)).sum() / 2
    L = (m * np.cross(a[:3].T, a[3:].T).T).sum(1)
    s = dict(zip(("x", "y", "z", "vx", "vy", "vz"), [a[k].astype(np.float64) for k in range(6)]))
    s["m"] = m.astype(np.float64)
    got = orc.diag(s, 1.2, 0.05)
    assert abs(got["W"] - float(W)) < 2e-15 * abs(float(W))
    assert abs(got["K"] - float(K)) < 2e-15 * abs(float(K))
    for c, k in enumerate(("Lx", "Ly", "Lz")):
        assert abs(got[k] - float(L[c])) < 1e-15


def test_plummer_energy_and_virial(orc):
    # E = -3 pi G M^2 / (64 a) for the Plummer model; virial 2K/|W| = 1.
    # Tolerances cover the sampling scatter of N = 4096 (seeds 1-5 span
    # E in [-0.154, -0.144] and 2K/|W| in [0.983, 1.013]).
    p = wl.plummer(4096, 1)
    d = orc.diag(p, 1.0, 0.01)
    assert abs(d["E"] / (-3 * math.pi / 64) - 1) < 0.06
    assert abs(2 * d["K"] / abs(d["W"]) - 1) < 0.03
