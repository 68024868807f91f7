"""Runtime properties on the GPU: checkpoint/resume continues bitwise, the
single-system step can be captured into a HIP graph and replayed (with eager
work and synchronisations between replays), kernel timing is recorded, and
the autotuner returns a valid plan."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

K = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_checkpoint_resume_bitwise(nb, ctx, tmp_path, prec):
    from paper_1803_01190_amd import checkpoint
    ic = wl.exp_disk(3000, 31)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    a = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, a, prm)
    nb.nbody_step_kdk(ctx, a, prm, 1e-3, 10)
    b = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, b, prm)
    nb.nbody_step_kdk(ctx, b, prm, 1e-3, 4)
    path = str(tmp_path / "snap.npz")
    checkpoint.save(path, b, prm, t=4e-3, step=4)
    del b
    c, prm2, t, step, _ = checkpoint.load(path)
    assert step == 4 and prm2 == prm
    nb.nbody_step_kdk(ctx, c, prm2, 1e-3, 6)
    torch.cuda.synchronize()
    for k in K:
        assert torch.equal(a[k], c[k]), k


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_checkpoint_resume_hermite_bitwise(nb, ctx, tmp_path, prec):
    # the Hermite scheme carries a and j of the last predicted state: a
    # snapshot holds the jerks too, and the resumed run continues bit for bit
    from paper_1803_01190_amd import checkpoint
    print(f"[case] hermite resume {prec}", flush=True)
    ic = wl.exp_disk(3000, 33)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    a = nb.System.from_arrays(ic)
    nb.nbody_accel_jerk(ctx, a, prm)
    nb.nbody_step_hermite(ctx, a, prm, 1e-3, 10)
    b = nb.System.from_arrays(ic)
    nb.nbody_accel_jerk(ctx, b, prm)
    nb.nbody_step_hermite(ctx, b, prm, 1e-3, 4)
    path = str(tmp_path / "snap_h.npz")
    checkpoint.save(path, b, prm, t=4e-3, step=4)
    del b
    c, prm2, t, step, _ = checkpoint.load(path)
    assert step == 4 and prm2 == prm
    nb.nbody_step_hermite(ctx, c, prm2, 1e-3, 6)
    torch.cuda.synchronize()
    for k in K + ("jx", "jy", "jz"):
        assert torch.equal(a[k], c[k]), k


@pytest.mark.parametrize("scheme", ["kdk", "o4"])
def test_single_system_graph_capture(nb, ctx, scheme):
    ic = wl.plummer(5000, 32)
    prm = nb.Params(eps=0.01, prec=nb.NB_MIXED)
    step = nb.nbody_step_kdk if scheme == "kdk" else nb.nbody_step_o4
    eager = nb.System.from_arrays(ic)
    cap = nb.System.from_arrays(ic)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for sys in (eager, cap):
            nb.nbody_accel(ctx, sys, prm, stream=s)
        step(ctx, cap, prm, 1e-3, 1, stream=s)    # warm-up: scratch is allocated here
        step(ctx, eager, prm, 1e-3, 1, stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step(ctx, cap, prm, 1e-3, 2, stream=s)
    for rep in range(4):
        g.replay()
        step(ctx, eager, prm, 1e-3, 2)
        junk = torch.randn(4096, device="cuda").cumsum(0)  # unrelated eager work
        torch.cuda.synchronize()
        for k in K:
            assert torch.equal(eager[k], cap[k]), (scheme, rep, k)
    del junk


def test_profile_counts_launches(nb, ctx):
    ic = wl.plummer(4096, 33)
    prm = nb.Params(eps=0.01, prec=nb.NB_FP64)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, s, prm)
    nb.nbody_profile_read(ctx)
    nb.nbody_profile_enable(ctx, True)
    nb.nbody_step_kdk(ctx, s, prm, 1e-3, 3)
    nb.nbody_profile_enable(ctx, False)
    p = nb.nbody_profile_read(ctx)
    assert p["accel_launches"] == 3 and p["update_launches"] == 3
    assert p["interactions"] == 3 * 4096 * 4096 and p["accel_ms"] > 0
    assert nb.nbody_profile_read(ctx)["accel_launches"] == 0  # read resets


def test_autotune_returns_a_valid_plan(nb, ctx, orc):
    n = 3000
    plan = nb.nbody_autotune(ctx, nb.NB_FP64, n, 200.0)
    assert plan["R"] in (1, 2, 4) and plan["block"] in (128, 256) and plan["split"] >= 1
    assert nb.nbody_plan_get(ctx, nb.NB_FP64, n) == plan
    ic = wl.plummer(n, 34)
    s = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, s, nb.Params(eps=0.01))
    ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, 0.01, want_scale=True)
    got = s.numpy()
    d = np.sqrt((got["ax"] - ax) ** 2 + (got["ay"] - ay) ** 2 + (got["az"] - az) ** 2)
    assert np.max(d / A) <= 1e-12
    nb.nbody_plan_set(ctx, nb.NB_FP64, n, None)
    # the float32 path never splits its running sum, whatever the plan says
    nb.nbody_plan_set(ctx, nb.NB_FP32, n, {"R": 2, "block": 128, "split": 8, "jsrc": 0})
    assert nb.nbody_plan_get(ctx, nb.NB_FP32, n)["split"] == 1
    nb.nbody_plan_set(ctx, nb.NB_FP32, n, None)


def test_plan_classes(nb, ctx, orc):
    # potential-pass and jerk plans are pinned separately from the
    # acceleration plan and change nothing beyond rounding
    n = 3000
    ic = wl.plummer(n, 35)
    prm = nb.Params(eps=0.01)
    pot = nb.NB_FP64 | nb.NB_PLAN_POTENTIAL
    jerk = nb.NB_FP64 | nb.NB_PLAN_JERK
    accel_plan = nb.nbody_plan_get(ctx, nb.NB_FP64, n)
    ref = orc.diag(ic, eps=0.01)
    ax, ay, az, jx, jy, jz, A, J = orc.accel_jerk(ic, 1.0, 0.01, want_scale=True)
    for pp in ({"R": 2, "block": 256, "split": 2, "jsrc": 1}, {"R": 1, "block": 256, "split": 1, "jsrc": 0}):
        nb.nbody_plan_set(ctx, pot, n, pp)
        assert nb.nbody_plan_get(ctx, pot, n) == pp
        assert nb.nbody_plan_get(ctx, nb.NB_FP64, n) == accel_plan
        s = nb.System.from_arrays(ic)
        d = nb.diag_dict(nb.nbody_diag(ctx, s, prm))
        assert abs(d["W"] - ref["W"]) <= 1e-12 * abs(ref["W"]), pp
    for jp in ({"R": 1, "block": 256, "split": 4, "jsrc": 0}, {"R": 2, "block": 256, "split": 1, "jsrc": 0}):
        nb.nbody_plan_set(ctx, jerk, n, jp)
        assert nb.nbody_plan_get(ctx, jerk, n) == jp
        s = nb.System.from_arrays(ic)
        nb.nbody_accel_jerk(ctx, s, prm)
        torch.cuda.synchronize()
        g = s.numpy()
        dj = np.sqrt((g["jx"] - jx) ** 2 + (g["jy"] - jy) ** 2 + (g["jz"] - jz) ** 2)
        assert np.max(dj / J) <= 1e-12, jp
    for bad_code, bad in ((jerk, {"R": 2, "block": 256, "split": 1, "jsrc": 1}),
                          (jerk, {"R": 4, "block": 256, "split": 1, "jsrc": 0}),
                          (pot, {"R": 2, "block": 128, "split": 1, "jsrc": 0}),
                          (nb.NB_FP64 | 0x400, {"R": 1, "block": 256, "split": 1, "jsrc": 0}),
                          (nb.NB_MIXED | nb.NB_PLAN_BATCH, {"R": 4, "block": 256, "split": 1, "jsrc": 0}),
                          (nb.NB_MIXED | nb.NB_PLAN_BATCH, {"R": 1, "block": 256, "split": 1, "jsrc": 1}),
                          # spatially ordered plans: mixed accelerations only, 256 lanes, R 1 or 2
                          (nb.NB_FP64, {"R": 1, "block": 256, "split": 1, "jsrc": 3}),
                          (nb.NB_FP32, {"R": 1, "block": 256, "split": 1, "jsrc": 2}),
                          (nb.NB_MIXED, {"R": 4, "block": 256, "split": 1, "jsrc": 3}),
                          (nb.NB_MIXED, {"R": 1, "block": 128, "split": 1, "jsrc": 2}),
                          (nb.NB_MIXED, {"R": 1, "block": 256, "split": 1, "jsrc": 6}),
                          (nb.NB_MIXED | nb.NB_PLAN_JERK, {"R": 1, "block": 256, "split": 1, "jsrc": 4}),
                          (nb.NB_MIXED | nb.NB_PLAN_POTENTIAL, {"R": 1, "block": 256, "split": 1, "jsrc": 3}),
                          (nb.NB_MIXED | nb.NB_PLAN_JERK, {"R": 1, "block": 256, "split": 1, "jsrc": 3}),
                          (nb.NB_FP64 | nb.NB_PLAN_JERK, {"R": 1, "block": 256, "split": 1, "jsrc": 2})):
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_plan_set(ctx, bad_code, n, bad)
        assert ei.value.status == nb.NB_EINVAL
    for code in (pot, jerk):
        tuned = nb.nbody_autotune(ctx, code, n, 100.0)
        assert tuned["block"] == 256 and tuned["R"] in (1, 2)
        assert nb.nbody_plan_get(ctx, code, n) == tuned
        nb.nbody_plan_set(ctx, code, n, None)


def test_autotune_with_spatial_plan_pinned(nb, ctx):
    # a pinned spatially ordered plan is the first candidate; autotuning its
    # key times whole systems and pins what it returns
    for n, plan in ((40000, {"R": 1, "block": 256, "split": 4, "jsrc": 3}),
                    (3000, {"R": 2, "block": 256, "split": 2, "jsrc": 2})):
        print(f"[case] autotune n={n} pinned {plan}", flush=True)
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, plan)
        try:
            tuned = nb.nbody_autotune(ctx, nb.NB_MIXED, n, 50.0)
            assert nb.nbody_plan_get(ctx, nb.NB_MIXED, n) == tuned
        finally:
            nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)


def _rate(nb, ctx, s, prm, plan, reps=6):
    nb.nbody_plan_set(ctx, prm.prec, s.n, plan)
    nb.nbody_accel(ctx, s, prm)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        nb.nbody_accel(ctx, s, prm)
    b.record()
    torch.cuda.synchronize()
    return reps * float(s.n) ** 2 / (a.elapsed_time(b) * 1e-3)


def test_autotune_finds_the_headline_plan_class(nb, ctx, orc):
    # tuning the N = 2^17 disk from the heuristic plan, over every candidate
    # on the whole system: the result sums in spatial order, matches the
    # oracle, and is within 3% of the committed plan's rate
    from oracle.metrics import force_errors
    n = 1 << 17
    print(f"[case] autotune mixed disk n={n}", flush=True)
    ic = wl.exp_disk(n, 2)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    committed = nb.read_plans()["mixed"]["17"]
    s = nb.System.from_arrays(ic)
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)
    try:
        tuned = nb.nbody_autotune_sys(ctx, nb.NB_MIXED, s, prm, 0.0)
        print(f"[tune] 2^17 mixed: tuned {tuned}, committed {committed}", flush=True)
        assert tuned["jsrc"] in (2, 3, 4, 5), tuned
        assert nb.nbody_plan_get(ctx, nb.NB_MIXED, n) == tuned
        rows = np.sort(np.random.default_rng(8).choice(n, size=512, replace=False))
        ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, 0.02, rows=rows, want_scale=True)
        hx, hy, hz = orc.halo_accel(ic["x"][rows], ic["y"][rows], ic["z"][rows], orc.Halo(h.v2, h.rc))
        A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
        rt = torch.as_tensor(rows, device="cuda")
        got = torch.stack([s[k][rt] for k in ("ax", "ay", "az")]).cpu().numpy()
        e = force_errors(got, np.stack([ax + hx, ay + hy, az + hz]), A)
        assert e["eps_cond"] <= 2e-7 and e["eps_rms"] <= 2e-7, e
        r_tuned = max(_rate(nb, ctx, s, prm, tuned) for _ in range(2))
        r_comm = max(_rate(nb, ctx, s, prm, committed) for _ in range(2))
        print(f"[tune] rates tuned {r_tuned:.4e} committed {r_comm:.4e}", flush=True)
        assert r_tuned >= 0.97 * r_comm, (tuned, r_tuned, committed, r_comm)
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)


def test_batch_autotune(nb, ctx):
    # the batch tuner times batch plans on the caller's state and sets and
    # pins the fastest; the batch then runs under it
    mix = wl.batch_mix(32, 5)
    off = mix["off"]
    B = len(off) - 1
    h = wl.default_halo()
    prms = [nb.Params(eps=0.01 if mix["kind"][k] == "plummer" else 0.02, prec=nb.NB_MIXED,
                      halo=mix["kind"][k] == "disk", halo_v2=h.v2, halo_rc=h.rc) for k in range(B)]
    b = nb.nbody_batch_create(ctx, off, prms, [1e-3] * B)
    try:
        s = nb.System.from_arrays(mix)
        best = nb.nbody_batch_autotune(ctx, b, s, 0.0)
        print(f"[tune] batch of {B}: {best}", flush=True)
        assert nb.nbody_batch_get_plan(ctx, b) == best
        nmax = int(np.diff(off).max())
        assert nb.nbody_plan_get(ctx, nb.NB_MIXED | nb.NB_PLAN_BATCH, nmax) == best
        got = {k: s[k].clone() for k in ("ax", "ay", "az")}
        nb.nbody_accel_batched(ctx, b, s)
        torch.cuda.synchronize()
        for k in ("ax", "ay", "az"):
            assert torch.equal(got[k], s[k]), k
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED | nb.NB_PLAN_BATCH, int(np.diff(off).max()), None)
        nb.nbody_batch_destroy(ctx, b)
