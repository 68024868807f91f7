"""Checks of the seeded input generators (not of the method)."""
import math

import numpy as np

import workloads as wl


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 seeded with 0 (the published reference)
    assert wl.splitmix64_reference(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                             0x06C45D188009454F]
    assert [int(v) for v in wl.Stream(0).u64(3)] == wl.splitmix64_reference(0, 3)
    s = wl.Stream(123)
    a = s.u64(5)
    b = s.u64(4)
    assert [int(v) for v in np.concatenate([a, b])] == wl.splitmix64_reference(123, 9)
    u = wl.Stream(5).uniform(100000)
    assert u.min() > 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.005


def test_plummer_radial_cdf_and_frame():
    n = 20000
    p = wl.plummer(n, 1)
    r = np.sort(np.sqrt(p["x"] ** 2 + p["y"] ** 2 + p["z"] ** 2))
    cdf = r ** 3 / (r ** 2 + 1) ** 1.5
    emp = (np.arange(n) + 0.5) / n
    assert np.max(np.abs(cdf - emp)) < 1.63 / math.sqrt(n)  # KS at 1%
    for k in ("x", "vx", "vz"):
        assert abs(np.sum(p["m"] * p[k])) < 1e-12
    # isotropic velocity dispersion: <v^2> = 3 pi / 32... total K = 3 pi / 64
    K = 0.5 * np.sum(p["m"] * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2))
    assert abs(K / (3 * math.pi / 64) - 1) < 0.03


def test_disk_profiles():
    n = 40000
    d = wl.exp_disk(n, 3)
    R = np.sqrt(d["x"] ** 2 + d["y"] ** 2)
    assert R.max() < 4.02
    # radial CDF of the truncated exponential
    Rs = np.sort(R)
    cdf = (1 - (1 + Rs) * np.exp(-Rs)) / (1 - 5 * math.exp(-4))
    assert np.max(np.abs(cdf - (np.arange(n) + 0.5) / n)) < 2.0 / math.sqrt(n) + 0.01
    # sech^2 vertical profile: CDF (1 + tanh(z/z0))/2
    zs = np.sort(d["z"])
    cz = 0.5 * (1 + np.tanh(zs / 0.1))
    assert np.max(np.abs(cz - (np.arange(n) + 0.5) / n)) < 2.0 / math.sqrt(n) + 0.01
    # the disk rotates: mean v_phi > 0 and L_z > 0
    vphi = (d["x"] * d["vy"] - d["y"] * d["vx"]) / np.maximum(R, 1e-12)
    assert np.mean(vphi) > 0.3


def test_kepler_pair_and_solver():
    k = wl.kepler_pair()
    assert np.sum(k["m"] * k["x"]) == 0 and np.sum(k["m"] * k["vy"]) == 0
    x, y = wl.kepler_relative_position(0.0)
    assert abs(x - 0.5) < 1e-15 and abs(y) < 1e-15
    x, y = wl.kepler_relative_position(math.pi)  # half period: apocentre
    assert abs(x + 1.5) < 1e-12 and abs(y) < 1e-12


def test_batch_and_requests():
    sizes = wl.batch_sizes(256, 4)
    assert sizes.min() >= 1024 and sizes.max() <= 65536
    b = wl.batch_mix(6, 4, 6, 8)
    assert b["off"][-1] == b["x"].size and len(b["kind"]) == 6
    reqs = wl.request_stream(50, 5, rate=2.0)
    t = [r["t_arrive"] for r in reqs]
    assert all(t2 > t1 for t1, t2 in zip(t, t[1:]))
    assert all(4096 <= r["n"] <= 1 << 20 and 10 <= r["steps"] <= 1000 for r in reqs)
