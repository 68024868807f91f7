"""GPU acceleration-and-jerk sum, fourth-order Hermite and RK4 steps against
the oracle, through the C ABI.

Gates: float64 a and j within 1e-12 of the oracle in the conditioned
measure (error over the sum of the terms' magnitudes); mixed 2e-6 (measured
at these sizes, every plan: at most 5.7e-7 for a and j) and float32 1e-3.
Integrated states are compared with the oracle's run of the same steps."""
import math

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 2e-6, "fp32": 1e-3}


def cond_err(got, ref, scale):
    d = np.sqrt(sum((g - r) ** 2 for g, r in zip(got, ref)))
    e = float(np.max(d / scale))
    print(f"[err] cond {e:.3e}", flush=True)
    return e


def gpu_aj(nb, ctx, ic, prm):
    s = nb.System.from_arrays(ic)
    nb.nbody_accel_jerk(ctx, s, prm)
    torch.cuda.synchronize()
    g = s.numpy()
    return (g["ax"], g["ay"], g["az"]), (g["jx"], g["jy"], g["jz"])


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("n", [1, 2, 17, 257, 1021, 4099])
def test_accel_jerk(nb, ctx, orc, prec, n):
    print(f"[case] accel_jerk {prec} n={n}", flush=True)
    ic = wl.plummer(n, 200 + n)
    prm = nb.Params(eps=0.01, prec=nb.PREC[prec])
    a, j = gpu_aj(nb, ctx, ic, prm)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.01, want_scale=True)
    if n == 1:
        assert all(np.all(v == 0) for v in (*a, *j))
        return
    assert cond_err(a, (ax, ay, az), A) <= TOL[prec]
    assert cond_err(j, (jx, jy, jz), J) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_accel_jerk_disk_with_halo(nb, ctx, orc, prec):
    print(f"[case] accel_jerk disk+halo {prec}", flush=True)
    ic = wl.exp_disk(3001, 201)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    a, j = gpu_aj(nb, ctx, ic, prm)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.02, orc.Halo(h.v2, h.rc), want_scale=True)
    # the halo terms join the scale: the halo's own a and j magnitudes
    hx, hy, hz = orc.halo_accel(ic["x"], ic["y"], ic["z"], orc.Halo(h.v2, h.rc))
    A = A + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
    _, _, _, hjx, hjy, hjz = orc.accel_jerk({**ic, "m": np.zeros(3001)}, 1.0, 0.02, orc.Halo(h.v2, h.rc))
    J = J + np.sqrt(hjx ** 2 + hjy ** 2 + hjz ** 2)
    assert cond_err(a, (ax, ay, az), A) <= TOL[prec]
    assert cond_err(j, (jx, jy, jz), J) <= TOL[prec]


def test_coincident_pair_without_softening(nb, ctx, orc):
    # eps = 0: a coincident pair contributes nothing (the oracle's reading)
    ic = wl.plummer(300, 202)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        ic[k][5] = ic[k][9]
    prm = nb.Params(eps=0.0, prec=nb.NB_FP64)
    a, j = gpu_aj(nb, ctx, ic, prm)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.0, want_scale=True)
    assert np.all(np.isfinite(np.concatenate([*a, *j])))
    assert cond_err(a, (ax, ay, az), A) <= 1e-12 and cond_err(j, (jx, jy, jz), J) <= 1e-12


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-160), ("mixed", 1e-25)])
def test_tiny_softening_jerk(nb, ctx, orc, prec, eps):
    # a softening whose square is not normal: the self pair drops out
    ic = wl.plummer(700, 209)
    a, j = gpu_aj(nb, ctx, ic, nb.Params(eps=eps, prec=nb.PREC[prec]))
    assert np.all(np.isfinite(np.concatenate([*a, *j])))
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, eps, want_scale=True)
    assert cond_err(a, (ax, ay, az), A) <= TOL[prec] and cond_err(j, (jx, jy, jz), J) <= TOL[prec]


def run_steps(nb, ctx, ic, prm, scheme, dt, steps):
    s = nb.System.from_arrays(ic)
    if scheme == "hermite":
        nb.nbody_accel_jerk(ctx, s, prm)
        nb.nbody_step_hermite(ctx, s, prm, dt, steps)
    else:
        nb.nbody_accel(ctx, s, prm)
        nb.nbody_step_rk4(ctx, s, prm, dt, steps)
    torch.cuda.synchronize()
    return s.numpy()


def oracle_steps(orc, ic, eps, halo, scheme, dt, steps):
    ref = orc.State(ic, eps=eps, halo=halo)
    if scheme == "hermite":
        ref.init_jerk()
        ref.step_hermite(dt, steps)
    else:
        ref.step_rk4(dt, steps)
    return ref


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
@pytest.mark.parametrize("model", ["plummer", "disk"])
def test_steps_match_oracle_fp64(nb, ctx, orc, scheme, model):
    print(f"[case] {scheme} fp64 {model}", flush=True)
    n, steps, dt = 2000, 6, 2e-3
    if model == "plummer":
        ic, eps, halo, prm = wl.plummer(n, 203), 0.01, None, nb.Params(eps=0.01)
    else:
        h = wl.default_halo()
        ic, eps, halo = wl.exp_disk(n, 204), 0.02, orc.Halo(h.v2, h.rc)
        prm = nb.Params(eps=eps, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    got = run_steps(nb, ctx, ic, prm, scheme, dt, steps)
    ref = oracle_steps(orc, ic, eps, halo, scheme, dt, steps)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-13 * np.max(np.abs(ref[k])), k
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-12 * np.max(np.abs(ref[k])), k
    for k in ("ax", "ay", "az") + (("jx", "jy", "jz") if scheme == "hermite" else ()):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-11 * np.max(np.abs(ref[k])), k


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_steps_reduced_precision(nb, ctx, orc, scheme, prec):
    print(f"[case] {scheme} {prec}", flush=True)
    n, steps, dt = 2000, 6, 2e-3
    ic = wl.plummer(n, 205)
    got = run_steps(nb, ctx, ic, nb.Params(eps=0.01, prec=nb.PREC[prec]), scheme, dt, steps)
    ref = oracle_steps(orc, ic, 0.01, None, scheme, dt, steps)
    # mixed keeps float64 state: position error ~ steps dt^2 |delta a|; float32
    # also rounds the state to float32 every step (~u |x| each)
    for k in ("x", "y", "z"):
        tol = 1e-9 if prec == "mixed" else 1e-5 * np.max(np.abs(ref[k]))
        assert np.max(np.abs(got[k] - ref[k])) <= tol, k


@pytest.mark.parametrize("scheme", ["hermite", "rk4"])
def test_kepler_fourth_order_on_gpu(nb, ctx, scheme):
    # the two-body orbit (e = 0.5, period 2 pi) with no softening: the
    # position error at t = 0.3 T falls ~16x when the step halves
    errs = []
    T = 2 * math.pi
    for count in (200, 400):
        got = run_steps(nb, ctx, wl.kepler_pair(), nb.Params(eps=0.0), scheme, 0.3 * T / count, count)
        ex, ey = wl.kepler_relative_position(0.3 * T)
        errs.append(math.hypot(got["x"][1] - got["x"][0] - ex, got["y"][1] - got["y"][0] - ey))
    assert 3.6 < math.log2(errs[0] / errs[1]) < 4.4, errs
    assert errs[1] < 1e-5


def test_rk4_potential_and_validation(nb, ctx, orc):
    ic = wl.plummer(1500, 206)
    s = nb.System.from_arrays(ic, with_phi=True)
    prm = nb.Params(eps=0.01)
    nb.nbody_accel(ctx, s, prm)
    nb.nbody_step_rk4(ctx, s, prm, 1e-3, 2)
    torch.cuda.synchronize()
    g = s.numpy()
    _, _, _, phi, A = orc.accel(g["x"], g["y"], g["z"], g["m"], 1.0, 0.01, want_phi=True, want_scale=True)
    assert np.max(np.abs(g["phi"] - phi) / np.abs(phi)) <= 1e-12
    with pytest.raises(nb.NBodyError) as ei:
        nb.nbody_step_rk4(ctx, s, prm, 1e-3, -1)
    assert ei.value.status == nb.NB_EINVAL
    with pytest.raises(nb.NBodyError) as ei:
        nb.nbody_step_hermite(ctx, s, prm, float("inf"), 1)
    assert ei.value.status == nb.NB_EINVAL
    cs, cp = s.c(), prm.c()
    st = nb._lib.nbody_accel_jerk(ctx, nb.ctypes.byref(cs), None, None, None, nb.ctypes.byref(cp), None)
    assert st == nb.NB_EINVAL


def test_hermite_zero_steps_and_empty(nb, ctx):
    s0 = nb.System(0)
    prm = nb.Params(eps=0.01)
    nb.nbody_accel_jerk(ctx, s0, prm)
    nb.nbody_step_hermite(ctx, s0, prm, 1e-3, 3)
    nb.nbody_step_rk4(ctx, s0, prm, 1e-3, 3)
    ic = wl.plummer(100, 207)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel_jerk(ctx, s, prm)
    before = s.numpy()
    nb.nbody_step_hermite(ctx, s, prm, 1e-3, 0)
    torch.cuda.synchronize()
    after = s.numpy()
    for k in before:
        assert np.array_equal(before[k], after[k])


# mixed jerk plans in spatial order (jsrc 2): far source tiles with tile-local
# float32 positions and velocities; the same gate as the other mixed plans
JERK_LOCAL = [dict(R=R, block=256, split=s, jsrc=2) for R in (1, 2) for s in (1, 3)]


def _aj_with_plan(nb, ctx, ic, prm, plan):
    code = nb.NB_MIXED | nb.NB_PLAN_JERK
    nb.nbody_plan_set(ctx, code, ic["x"].size, plan)
    try:
        return gpu_aj(nb, ctx, ic, prm)
    finally:
        nb.nbody_plan_set(ctx, code, ic["x"].size, None)


@pytest.mark.parametrize("plan", JERK_LOCAL, ids=lambda p: f"R{p['R']}s{p['split']}")
@pytest.mark.parametrize("model,n", [("plummer", 4099), ("disk", 20000), ("plummer", 300)])
def test_accel_jerk_spatial_order(nb, ctx, orc, plan, model, n):
    print(f"[case] accel_jerk mixed spatial order {model} n={n} plan={plan}", flush=True)
    if model == "disk":
        h = wl.default_halo()
        ic, eps = wl.exp_disk(n, 208), 0.02
        prm = nb.Params(eps=eps, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
        halo = orc.Halo(h.v2, h.rc)
    else:
        ic, eps, halo = wl.plummer(n, 209), 0.01, None
        prm = nb.Params(eps=eps, prec=nb.NB_MIXED)
    a, j = _aj_with_plan(nb, ctx, ic, prm, plan)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, eps, halo, want_scale=True)
    if halo is not None:
        # the halo terms join the scale: the halo's own a and j magnitudes
        hx, hy, hz = orc.halo_accel(ic["x"], ic["y"], ic["z"], halo)
        A = A + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
        _, _, _, hjx, hjy, hjz = orc.accel_jerk({**ic, "m": np.zeros(n)}, 1.0, eps, halo)
        J = J + np.sqrt(hjx ** 2 + hjy ** 2 + hjz ** 2)
    assert cond_err(a, (ax, ay, az), A) <= TOL["mixed"]
    assert cond_err(j, (jx, jy, jz), J) <= TOL["mixed"]
    # and close to the plan that forms every separation in float64
    a0, j0 = _aj_with_plan(nb, ctx, ic, prm, dict(R=2, block=256, split=1, jsrc=0))
    assert cond_err(a, a0, A) <= TOL["mixed"] and cond_err(j, j0, J) <= TOL["mixed"]


@pytest.mark.parametrize("split", [1, 4])
def test_hermite_spatial_order_steps(nb, ctx, split):
    # Hermite steps under the spatially ordered jerk plan (corrector in the
    # pair kernel with split 1, in the reduction otherwise): deterministic,
    # and within the mixed force error of the steps under the jsrc 0 plan
    print(f"[case] hermite mixed spatial order split={split}", flush=True)
    n, steps, dt = 20000, 5, 1e-3
    ic = wl.exp_disk(n, 210)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    code = nb.NB_MIXED | nb.NB_PLAN_JERK
    local = {"R": 2, "block": 256, "split": split, "jsrc": 2}
    outs = []
    for plan in (local, local, {"R": 2, "block": 256, "split": 1, "jsrc": 0}):
        nb.nbody_plan_set(ctx, code, n, plan)
        try:
            outs.append(run_steps(nb, ctx, ic, prm, "hermite", dt, steps))
        finally:
            nb.nbody_plan_set(ctx, code, n, None)
    for k in ("x", "vx", "ax", "jx"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.max(np.abs(outs[0][k] - outs[2][k])) <= 1e-9 * np.max(np.abs(outs[2][k])), k


def test_jerk_spatial_order_edges(nb, ctx, orc):
    # eps = 0 with a coincident pair (self and coincident pairs drop out), and
    # a translated, boosted system (tile-local coordinates keep the accuracy)
    print("[case] jerk spatial order edges", flush=True)
    plan = dict(R=2, block=256, split=2, jsrc=2)
    ic = wl.plummer(3000, 211)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        ic[k][5] = ic[k][6]
    a, j = _aj_with_plan(nb, ctx, ic, nb.Params(eps=0.0, prec=nb.NB_MIXED), plan)
    assert np.all(np.isfinite(np.concatenate([*a, *j])))
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.0, want_scale=True)
    assert cond_err(a, (ax, ay, az), A) <= TOL["mixed"] and cond_err(j, (jx, jy, jz), J) <= TOL["mixed"]
    sh = dict(ic)
    sh["x"] = ic["x"] + 1000.0
    sh["vy"] = ic["vy"] + 50.0
    a2, j2 = _aj_with_plan(nb, ctx, sh, nb.Params(eps=0.01, prec=nb.NB_MIXED), plan)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.01, want_scale=True)
    assert cond_err(a2, (ax, ay, az), A) <= TOL["mixed"] and cond_err(j2, (jx, jy, jz), J) <= TOL["mixed"]
