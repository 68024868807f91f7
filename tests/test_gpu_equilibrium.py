"""Disk initial conditions iterated to the balance of Section 1, Eqs. (3)-(4)
with the library's own forces (paper_1803_01190_amd/equilibrium.py), against
the one-shot recipe they start from (rotation from the spherical enclosed
mass): the iterated disk keeps the recipe's radii, azimuths and masses, its
rotation follows the measured circular speed, and early in a run its surface
density profile drifts several times less (and its radial dispersion profile
no more)."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

EDGES = np.linspace(0.0, 4.0, 17)


def profiles(st):
    R = np.hypot(st["x"], st["y"])
    vR = (st["x"] * st["vx"] + st["y"] * st["vy"]) / np.maximum(R, 1e-300)
    b = np.clip(np.searchsorted(EDGES, R, side="right") - 1, 0, len(EDGES) - 2)
    m = np.bincount(b, weights=st["m"], minlength=len(EDGES) - 1)
    mv = np.bincount(b, weights=st["m"] * vR, minlength=len(EDGES) - 1) / m
    mv2 = np.bincount(b, weights=st["m"] * vR * vR, minlength=len(EDGES) - 1) / m
    return m, np.sqrt(np.maximum(mv2 - mv * mv, 0.0))


def drift(nb, ctx, ic, prm, dt, steps):
    m0, s0 = profiles(ic)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, s, prm)
    nb.nbody_step_kdk(ctx, s, prm, dt, steps)
    torch.cuda.synchronize()
    m1, s1 = profiles(s.numpy())
    inner = slice(1, 12)   # R in [0.25, 3): bins with many particles
    return {"sigma": float(np.abs(m1 - m0).sum() / m0.sum()),
            "sigma_R": float(np.mean(np.abs(s1[inner] - s0[inner]) / s0[inner]))}


@pytest.mark.parametrize("kind", ["disk_sg", "disk"])
def test_equilibrium_disk_drifts_less(nb, ctx, kind):
    from paper_1803_01190_amd.equilibrium import equilibrium_disk
    n = 1 << 15
    print(f"[case] equilibrium disk {kind} n={n}", flush=True)
    ic = wl.make(kind, n, 31)
    halo = None if kind == "disk_sg" else wl.default_halo()
    info = {}
    eq = equilibrium_disk(ctx, ic, halo=halo, seed=7, info=info)
    # same radii and azimuths up to the centre-of-mass shift, same masses
    assert np.array_equal(eq["m"], ic["m"])
    R0, R1 = np.hypot(ic["x"], ic["y"]), np.hypot(eq["x"], eq["y"])
    assert np.max(np.abs(R1 - R0)) <= 1e-2
    assert abs(float((eq["m"] * eq["vx"]).sum())) <= 1e-12 and abs(float((eq["m"] * eq["z"]).sum())) <= 1e-12
    # the measured circular speed has settled over the iterations
    vc = np.asarray(info["vc2"])
    assert np.max(np.abs(vc[-1] - vc[-2])) <= 0.05 * np.max(np.abs(vc[-1]))
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=halo is not None,
                    halo_v2=halo.v2 if halo else 0.0, halo_rc=halo.rc if halo else 0.0)
    d_recipe = drift(nb, ctx, ic, prm, 0.01, 300)
    d_eq = drift(nb, ctx, eq, prm, 0.01, 300)
    print(f"[drift] {kind}: recipe {d_recipe}, iterated {d_eq}", flush=True)
    # measured at t = 3: the surface-density profile moves about 7x (paper's
    # self-gravitating disk) and 9x (with the halo) less; the radial
    # dispersion, which the Q = 1.2 disk's own instability heats, drifts 10%
    # less without the halo and about the same (within 10%) with it, where the
    # halo already sets most of the rotation
    assert d_eq["sigma"] < 0.5 * d_recipe["sigma"], (d_eq, d_recipe)
    if kind == "disk_sg":
        assert d_eq["sigma_R"] < d_recipe["sigma_R"], (d_eq, d_recipe)
    else:
        assert d_eq["sigma_R"] < 1.25 * d_recipe["sigma_R"], (d_eq, d_recipe)
