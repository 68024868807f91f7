"""nbody_accel_static, the acceleration entry point that allocates nothing
(its scratch is a static device array), against nbody_accel through the C
ABI: bitwise when the plan's split fits the static scratch, within the
precision's gate (conditioned by the oracle's sum of |f|) when the split had
to shrink, and a clear NB_EINVAL for sizes beyond the static maximum.  Calls
follow each other on one GPU, so each one must not depend on what the
previous one left in the shared array."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.metrics import force_errors

pytestmark = pytest.mark.gpu

SPATIAL = {"R": 1, "block": 256, "split": 4, "jsrc": 3}


def both(nb, ctx, ic, prm):
    a = nb.System.from_arrays(ic)
    b = nb.System.from_arrays(ic)
    nb.nbody_accel(ctx, a, prm)
    nb.nbody_accel_static(ctx, b, prm)
    torch.cuda.synchronize()
    return a, b


def test_two_calls_in_a_row_bitwise(nb, ctx):
    # first a larger system, then a smaller one: the second call runs over
    # what the first left in the static array
    h = wl.default_halo()
    cases = [(40000, "mixed", SPATIAL), (3001, "mixed", SPATIAL),
             (5000, "fp64", {"R": 2, "block": 256, "split": 8, "jsrc": 1}),
             (1500, "fp32", None)]
    for n, prec, plan in cases:
        print(f"[case] static accel n={n} {prec} plan={plan}", flush=True)
        ic = wl.exp_disk(n, 40 + n % 7)
        prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
        if plan is not None:
            nb.nbody_plan_set(ctx, nb.PREC[prec], n, plan)
        try:
            a, b = both(nb, ctx, ic, prm)
        finally:
            if plan is not None:
                nb.nbody_plan_set(ctx, nb.PREC[prec], n, None)
        for k in ("ax", "ay", "az"):
            assert torch.equal(a[k], b[k]), (n, prec, k)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_split_shrinks_to_fit(nb, ctx, orc, prec):
    # N = 2^19 disk under a 32-way split: the partial sums (512 MiB) do not
    # fit, the static call sums in 4 chunks; both results meet the gate
    # against the oracle on sampled rows, and each other
    n = 1 << 19
    print(f"[case] static accel n={n} {prec} split shrinks", flush=True)
    plan = {**SPATIAL, "split": 32} if prec == "mixed" else {"R": 2, "block": 256, "split": 32, "jsrc": 1}
    gate = {"mixed": 2e-7, "fp64": 1e-12}[prec]
    ic = wl.exp_disk(n, 2)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
    nb.nbody_plan_set(ctx, nb.PREC[prec], n, plan)
    try:
        a, b = both(nb, ctx, ic, prm)
    finally:
        nb.nbody_plan_set(ctx, nb.PREC[prec], n, None)
    rows = np.sort(np.random.default_rng(5).choice(n, size=256, replace=False))
    ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, 0.02, rows=rows, want_scale=True)
    hx, hy, hz = orc.halo_accel(ic["x"][rows], ic["y"][rows], ic["z"][rows], orc.Halo(h.v2, h.rc))
    ref = np.stack([ax + hx, ay + hy, az + hz])
    A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
    rt = torch.as_tensor(rows, device="cuda")
    ga = torch.stack([a[k][rt] for k in ("ax", "ay", "az")]).cpu().numpy()
    gb = torch.stack([b[k][rt] for k in ("ax", "ay", "az")]).cpu().numpy()
    for got in (ga, gb):
        e = force_errors(got, ref, A)
        assert e["eps_cond"] <= gate and e["eps_rms"] <= gate, (prec, e)
    assert force_errors(gb, ga, A)["eps_cond"] <= gate


def test_rejects_size_beyond_static_maximum(nb, ctx):
    # a spatially ordered plan needs about 56 B per particle of order
    # scratch: 2.5e6 particles exceed the 128 MiB array; nothing is launched
    n = 2_500_000
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, {**SPATIAL, "split": 1})
    try:
        ic = {k: np.linspace(0.0, 1.0, n) for k in ("x", "y", "z")}
        ic["m"] = np.full(n, 1.0 / n)
        s = nb.System.from_arrays(ic)
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_accel_static(ctx, s, nb.Params(eps=0.02, prec=nb.NB_MIXED))
        assert ei.value.status == nb.NB_EINVAL and "static scratch" in str(ei.value)
        assert not s["ax"].any()
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)
