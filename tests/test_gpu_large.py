"""Full-size parity: the N = 2^20 exponential disk (eps = 0.02, halo) in the
launch configuration the benchmark times (plans from tuned_plans.json),
checked on rows the oracle computes one by one (each summed over all N
sources), plus the N = 2^17 disk with both integrators.

Stated errors (measured on sampled rows of this workload): mixed with the
tuned tile-local plans eps_rms 5.2e-8 to 5.4e-8 / eps_cond 4.2e-8 to 4.7e-8
(their far-tile separations carry up to a few u of relative error, against
u/2 when every separation is a rounded float64 difference, which gives
1.8e-8), gated at 2e-7; fp32 eps_rms 4.9e-4 / eps_cond 8.0e-4, gated at 2e-3; fp64 gated at
1e-12.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.metrics import force_errors

pytestmark = pytest.mark.gpu

GATE = {"fp64": 1e-12, "mixed": 2e-7, "fp32": 2e-3}


@pytest.fixture(scope="module")
def disk20():
    return wl.exp_disk(1 << 20, 2)


def oracle_rows(orc, ic, rows, eps, halo):
    ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, eps, rows=rows, want_scale=True)
    hx, hy, hz = orc.halo_accel(ic["x"][rows], ic["y"][rows], ic["z"][rows], orc.Halo(halo.v2, halo.rc))
    return np.stack([ax + hx, ay + hy, az + hz]), A + np.sqrt(hx * hx + hy * hy + hz * hz)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_disk_2p20_sampled(nb, ctx, orc, disk20, prec):
    n = 1 << 20
    print(f"[case] disk 2^20 {prec} sampled rows", flush=True)
    h = wl.default_halo()
    nb.load_plans(ctx)
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    s = nb.System.from_arrays(disk20)
    nb.nbody_accel(ctx, s, prm)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, size=512, replace=False))
    rt = torch.as_tensor(rows, device="cuda")
    got = torch.stack([s["ax"][rt], s["ay"][rt], s["az"][rt]]).cpu().numpy()
    ref, A = oracle_rows(orc, disk20, rows, 0.02, h)
    e = force_errors(got, ref, A)
    assert e["eps_rms"] <= GATE[prec] and e["eps_cond"] <= GATE[prec], (prec, e)
    # one KDK step in the timed configuration: the sampled positions follow
    # r + dt (v + dt/2 a) with the oracle's a
    dt = 1e-3
    nb.nbody_step_kdk(ctx, s, prm, dt, 1)
    x1 = s["x"][rt].cpu().numpy()
    want = disk20["x"][rows] + dt * (disk20["vx"][rows] + 0.5 * dt * ref[0])
    # float64 state: rounding of r plus dt^2/2 times the force error of the path
    tol = {"fp64": 1e-15, "mixed": 1e-13, "fp32": 1e-6}[prec]
    assert np.max(np.abs(x1 - want)) <= tol * np.max(np.abs(want)), prec
    # Newton's third law at full size: sum m a over all particles, without
    # the halo, is round-off of sum m A
    if prec == "fp64":
        prm0 = nb.Params(eps=0.02, prec=nb.NB_FP64)
        s2 = nb.System.from_arrays(disk20)
        nb.nbody_accel(ctx, s2, prm0)
        m = s2["m"]
        net = torch.stack([(m * s2[k]).sum() for k in ("ax", "ay", "az")]).abs().max().item()
        scale = float(np.sum(disk20["m"][rows] * A) * n / rows.size)
        assert net <= 1e-13 * scale, (net, scale)


# the quarter-tile forms (jsrc 4 and 5) at the sizes and splits of the tuned
# mixed plans, on the same sampled rows and gate
@pytest.mark.parametrize("log2n,plan", [(20, {"R": 1, "block": 256, "split": 32, "jsrc": 4}),
                                        (17, {"R": 2, "block": 256, "split": 16, "jsrc": 4}),
                                        (20, {"R": 1, "block": 256, "split": 16, "jsrc": 5})],
                         ids=["2p20R1s32", "2p17R2s16", "2p20R1s16j5"])
def test_disk_quarter_plan_sampled(nb, ctx, orc, disk20, log2n, plan):
    n = 1 << log2n
    print(f"[case] disk 2^{log2n} mixed quarter-tile plan {plan} sampled rows", flush=True)
    ic = disk20 if log2n == 20 else wl.exp_disk(n, 2)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    s = nb.System.from_arrays(ic)
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, plan)
    try:
        nb.nbody_accel(ctx, s, prm)
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)
    rng = np.random.default_rng(13)
    rows = np.sort(rng.choice(n, size=512, replace=False))
    rt = torch.as_tensor(rows, device="cuda")
    got = torch.stack([s["ax"][rt], s["ay"][rt], s["az"][rt]]).cpu().numpy()
    ref, A = oracle_rows(orc, ic, rows, 0.02, h)
    e = force_errors(got, ref, A)
    print(f"[err] 2^{log2n} quarter plan: {e}", flush=True)
    assert e["eps_rms"] <= GATE["mixed"] and e["eps_cond"] <= GATE["mixed"], e


# acceleration and jerk of the fourth-order Hermite scheme in the launch
# configuration the Hermite benchmark times (the tuned jerk plans: for mixed,
# the spatially ordered plan with R 1 and a 32-way split from N = 2^17 on)
JERK_GATE = {"fp64": (1e-12, 1e-12), "mixed": (2e-7, 5e-7), "fp32": (2e-3, 2e-3)}


@pytest.mark.parametrize("log2n", [17, 20])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_disk_jerk_sampled(nb, ctx, orc, disk20, prec, log2n):
    n = 1 << log2n
    print(f"[case] disk 2^{log2n} {prec} acceleration and jerk, sampled rows", flush=True)
    ic = disk20 if log2n == 20 else wl.exp_disk(n, 2)
    h = wl.default_halo()
    nb.load_plans(ctx)
    plan = nb.nbody_plan_get(ctx, nb.PREC[prec] | nb.NB_PLAN_JERK, n)
    if prec == "mixed":
        assert plan["jsrc"] == 2, plan  # the tuned plan is the one under test
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel_jerk(ctx, s, prm)
    rng = np.random.default_rng(12)
    rows = np.sort(rng.choice(n, size=512, replace=False))
    rt = torch.as_tensor(rows, device="cuda")
    got = torch.stack([s[k][rt] for k in ("ax", "ay", "az", "jx", "jy", "jz")]).cpu().numpy()
    halo = orc.Halo(h.v2, h.rc)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.02, halo, want_scale=True, rows=rows)
    # the halo's own a and j magnitudes join the scales
    sub = {k: ic[k][rows] for k in ("x", "y", "z", "vx", "vy", "vz")}
    _, _, _, hjx, hjy, hjz = orc.accel_jerk({**sub, "m": np.zeros(rows.size)}, 1.0, 0.02, halo)
    hx, hy, hz = orc.halo_accel(sub["x"], sub["y"], sub["z"], halo)
    A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
    J = J + np.sqrt(hjx * hjx + hjy * hjy + hjz * hjz)
    ea = force_errors(got[:3], np.stack([ax, ay, az]), A)
    ej = force_errors(got[3:], np.stack([jx, jy, jz]), J)
    print(f"[err] 2^{log2n} {prec} plan {plan}: a {ea}  j {ej}", flush=True)
    ga, gj = JERK_GATE[prec]
    assert ea["eps_cond"] <= ga and ea["eps_rms"] <= ga, ea
    assert ej["eps_cond"] <= gj, ej


@pytest.mark.parametrize("scheme", ["kdk", "o4"])
def test_disk_2p17_integrators_conserve(nb, ctx, scheme):
    # N = 2^17 disk: second- vs fourth-order.  L_z is conserved by both
    # schemes up to round-off in float64; energy drift follows the order.
    n = 1 << 17
    print(f"[case] disk 2^17 {scheme} fp64", flush=True)
    ic = wl.exp_disk(n, 3)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_FP64, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, s, prm)
    d0 = nb.diag_dict(nb.nbody_diag(ctx, s, prm))
    if scheme == "kdk":
        nb.nbody_step_kdk(ctx, s, prm, 1e-3, 20)
    else:
        nb.nbody_step_o4(ctx, s, prm, 1e-3, 20)
    d1 = nb.diag_dict(nb.nbody_diag(ctx, s, prm))
    assert abs(d1["Lz"] - d0["Lz"]) <= 1e-13 * abs(d0["Lz"])
    assert abs(d1["E"] - d0["E"]) <= 1e-6 * abs(d0["E"])
