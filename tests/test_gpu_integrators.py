"""GPU leapfrog (Eqs. (5)-(7)), fourth-order composition and conserved
quantities (Eqs. (8)-(10)) against the CPU oracle, through the C ABI.

Trajectories diverge exponentially, so the float64 trajectory gate is
self-calibrated: the GPU's distance from the oracle must stay within 10x
the distance between two oracle runs that differ only in the order of the
source sum (ascending vs descending j), over the same horizon.
"""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def gpu_run(nb, ctx, ic, prm, dt, nsteps, scheme="kdk", diag_every=0):
    s = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, s, prm)
    diags = []
    if diag_every:
        diags.append(nb.diag_dict(nb.nbody_diag(ctx, s, prm)))
    done = 0
    while done < nsteps:
        k = min(diag_every or nsteps, nsteps - done)
        if scheme == "kdk":
            nb.nbody_step_kdk(ctx, s, prm, dt, k)
        else:
            nb.nbody_step_o4(ctx, s, prm, dt, k)
        done += k
        if diag_every:
            diags.append(nb.diag_dict(nb.nbody_diag(ctx, s, prm)))
    torch.cuda.synchronize()
    return s.numpy(), diags


def orc_run(orc, ic, eps, dt, nsteps, scheme="kdk", reverse=False, halo=None, diag_every=0):
    st = orc.State(ic, eps=eps, reverse_j=reverse, halo=halo)
    diags = [st.diag()] if diag_every else []
    done = 0
    while done < nsteps:
        k = min(diag_every or nsteps, nsteps - done)
        (st.step_kdk if scheme == "kdk" else st.step_o4)(dt, k)
        done += k
        if diag_every:
            diags.append(st.diag())
    return st, diags


def maxdev(a, b, keys=("x", "y", "z")):
    return max(np.max(np.abs(a[k] - b[k])) for k in keys)


def test_kdk_plummer_4096_100_steps(nb, ctx, orc):
    # Plummer N = 4096, eps = 0.01, dt = 1e-3, 100 KDK steps, float64
    print("[case] kdk plummer 4096 x100 fp64", flush=True)
    ic = wl.plummer(4096, 1)
    eps, dt, n = 0.01, 1e-3, 100
    ref, dref = orc_run(orc, ic, eps, dt, n, diag_every=10)
    alt, _ = orc_run(orc, ic, eps, dt, n, reverse=True)
    got, dgot = gpu_run(nb, ctx, ic, nb.Params(eps=eps, prec=nb.NB_FP64), dt, n, diag_every=10)
    d_orc = maxdev(ref, alt)
    d_gpu = maxdev(got, ref)
    assert d_gpu <= 10 * d_orc + 1e-15, (d_gpu, d_orc)
    dv = maxdev(got, ref, ("vx", "vy", "vz"))
    dv_orc = maxdev(ref, alt, ("vx", "vy", "vz"))
    assert dv <= 10 * dv_orc + 1e-14, (dv, dv_orc)
    # E, P, L at every checkpoint
    pscale = np.sum(ic["m"] * np.sqrt(ic["vx"] ** 2 + ic["vy"] ** 2 + ic["vz"] ** 2))
    lscale = np.sum(ic["m"] * np.sqrt(ic["x"] ** 2 + ic["y"] ** 2 + ic["z"] ** 2)
                    * np.sqrt(ic["vx"] ** 2 + ic["vy"] ** 2 + ic["vz"] ** 2))
    for g, r in zip(dgot, dref):
        assert abs(g["E"] - r["E"]) <= 1e-12 * abs(r["E"]), (g["E"], r["E"])
        for k in ("Px", "Py", "Pz"):
            assert abs(g[k] - r[k]) <= 1e-12 * pscale
        for k in ("Lx", "Ly", "Lz"):
            assert abs(g[k] - r[k]) <= 1e-12 * lscale


def test_kdk_disk_with_halo(nb, ctx, orc):
    print("[case] kdk disk 3000 + halo x20 fp64", flush=True)
    ic = wl.exp_disk(3000, 2)
    h = wl.default_halo()
    eps, dt, n = 0.02, 1e-3, 20
    ref, dref = orc_run(orc, ic, eps, dt, n, halo=orc.Halo(h.v2, h.rc), diag_every=20)
    alt, _ = orc_run(orc, ic, eps, dt, n, reverse=True, halo=orc.Halo(h.v2, h.rc))
    prm = nb.Params(eps=eps, prec=nb.NB_FP64, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    got, dgot = gpu_run(nb, ctx, ic, prm, dt, n, diag_every=20)
    assert maxdev(got, ref) <= 10 * maxdev(ref, alt) + 1e-15
    for g, r in zip(dgot, dref):
        for k in ("E", "W", "Wext", "K", "Lz"):
            assert abs(g[k] - r[k]) <= 1e-12 * abs(r[k]), (k, g[k], r[k])


def test_o4_against_oracle(nb, ctx, orc):
    print("[case] o4 plummer 1024 x10 fp64", flush=True)
    ic = wl.plummer(1024, 3)
    eps, dt, n = 0.01, 2e-3, 10
    ref, _ = orc_run(orc, ic, eps, dt, n, scheme="o4")
    alt, _ = orc_run(orc, ic, eps, dt, n, scheme="o4", reverse=True)
    got, _ = gpu_run(nb, ctx, ic, nb.Params(eps=eps, prec=nb.NB_FP64), dt, n, scheme="o4")
    assert maxdev(got, ref) <= 10 * maxdev(ref, alt) + 1e-15


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-7), ("fp32", 1e-4)])
def test_reduced_precision_short_run(nb, ctx, orc, prec, tol):
    # 10 steps: positions move by ~1e-2; the force error (~1e-6 mixed,
    # ~1e-4 float32, relative) enters through dt^2 and state rounding
    print(f"[case] kdk {prec} plummer 2048 x10", flush=True)
    ic = wl.plummer(2048, 4)
    ref, _ = orc_run(orc, ic, 0.01, 1e-3, 10)
    got, _ = gpu_run(nb, ctx, ic, nb.Params(eps=0.01, prec=nb.PREC[prec]), 1e-3, 10)
    scale = np.max(np.abs(ref["x"]))
    assert maxdev(got, ref) <= tol * scale


def test_single_particle_and_zero_steps(nb, ctx):
    ic = {"x": [1.0], "y": [2.0], "z": [3.0], "vx": [0.5], "vy": [-0.25], "vz": [0.125], "m": [1.0]}
    got, _ = gpu_run(nb, ctx, ic, nb.Params(eps=0.1), 0.125, 64)
    # no force on a lone particle: x = x0 + v t exactly (dyadic values)
    assert got["x"][0] == 5.0 and got["y"][0] == 0.0 and got["z"][0] == 4.0
    s = nb.System.from_arrays(wl.plummer(50, 1))
    before = s["x"].clone()
    nb.nbody_step_kdk(ctx, s, nb.Params(eps=0.1), 1e-3, 0)
    torch.cuda.synchronize()
    assert torch.equal(before, s["x"])


@pytest.mark.parametrize("n", [1, 2, 300, 5000])
def test_diag_fp64(nb, ctx, orc, n):
    print(f"[case] diag n={n}", flush=True)
    ic = wl.plummer(n, 20 + n)
    h = wl.default_halo()
    for halo in (None, h):
        prm = nb.Params(eps=0.01)
        if halo:
            prm.halo, prm.halo_v2, prm.halo_rc = True, h.v2, h.rc
        s = nb.System.from_arrays(ic)
        for prec in (nb.NB_FP64, nb.NB_FP32):  # diagnostics are float64 in every mode
            prm.prec = prec
            g = nb.diag_dict(nb.nbody_diag(ctx, s, prm))
            r = orc.diag(ic, 1.0, 0.01, orc.Halo(h.v2, h.rc) if halo else None)
            for k in ("K", "W", "Wext", "E", "M"):
                assert abs(g[k] - r[k]) <= 1e-12 * max(abs(r[k]), 1e-300), (k, g[k], r[k])
            for k in ("Px", "Py", "Pz", "Lx", "Ly", "Lz", "Cx", "Cy", "Cz"):
                assert abs(g[k] - r[k]) <= 1e-14, (k, g[k], r[k])
