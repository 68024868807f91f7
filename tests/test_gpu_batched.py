"""Batched persistent launches: many independent systems in one launch.

Each system's result must be bitwise equal to the same system run alone
under the single-system plan the batch reports for it (its chunk count and,
for mixed systems in spatial order, its far-tile form), for several batch
plans; the HIP-graph replay must equal eager launches on every replay, and
every system must match the oracle (float64 gate 1e-12, mixed and float32
their own gates).
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.metrics import force_errors

pytestmark = pytest.mark.gpu

K = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")


def make_batch(specs):
    """specs: list of (kind, n, seed, eps, prec_name, halo_bool, dt)."""
    parts, off = [], [0]
    for kind, n, seed, *_ in specs:
        ic = wl.make(kind, n, seed) if n > 0 else {k: np.zeros(0) for k in wl.FIELDS}
        parts.append(ic)
        off.append(off[-1] + n)
    packed = {k: np.concatenate([p[k] for p in parts]) for k in wl.FIELDS}
    return packed, off, parts


def params_of(nb, spec):
    kind, n, seed, eps, prec, halo, dt = spec
    h = wl.default_halo()
    return nb.Params(eps=eps, prec=nb.PREC[prec], halo=halo, halo_v2=h.v2 if halo else 0.0,
                     halo_rc=h.rc if halo else 0.0)


SPECS = [
    ("plummer", 1000, 1, 0.01, "fp64", False, 1e-3),
    ("disk", 777, 2, 0.02, "fp64", True, 2e-3),
    ("plummer", 1, 3, 0.01, "fp64", False, 1e-3),
    ("plummer", 0, 4, 0.01, "fp64", False, 1e-3),
    ("plummer", 2, 5, 0.0, "fp64", False, 1e-3),
    ("disk", 3001, 6, 0.02, "mixed", True, 1e-3),
    ("plummer", 513, 7, 0.0, "mixed", False, 5e-4),
    ("plummer", 1300, 8, 0.01, "fp32", False, 1e-3),
    ("disk", 257, 9, 0.02, "fp32", True, 1e-3),
    ("plummer", 4099, 10, 0.01, "fp64", False, 1e-3),
]


def single(nb, ctx, ic, prm, plan, fn):
    s = nb.System.from_arrays(ic)
    if s.n == 0:
        return s.numpy()
    nb.nbody_plan_set(ctx, prm.prec, s.n, plan)
    try:
        fn(s)
        torch.cuda.synchronize()
    finally:
        nb.nbody_plan_set(ctx, prm.prec, s.n, None)
    return s.numpy()


# batch plans: R, source tiles per chunk (0: whole systems), jsrc of the mixed systems
BATCH_PLANS = [None,  # the default plan
               {"R": 1, "block": 256, "split": 0, "jsrc": 0},
               {"R": 2, "block": 256, "split": 2, "jsrc": 0},
               {"R": 1, "block": 256, "split": 3, "jsrc": 3},
               {"R": 2, "block": 256, "split": 1, "jsrc": 2},
               {"R": 2, "block": 256, "split": 3, "jsrc": 4},
               {"R": 1, "block": 256, "split": 2, "jsrc": 5}]


def plan_id(p):
    return "default" if p is None else f"R{p['R']}s{p['split']}j{p['jsrc']}"


@pytest.mark.parametrize("bplan", BATCH_PLANS, ids=plan_id)
def test_accel_batched_equals_single_and_oracle(nb, ctx, orc, bplan):
    print(f"[case] batched accel plan {bplan}", flush=True)
    packed, off, parts = make_batch(SPECS)
    prms = [params_of(nb, sp) for sp in SPECS]
    b = nb.nbody_batch_create(ctx, off, prms, [sp[6] for sp in SPECS])
    try:
        if bplan is not None:
            nb.nbody_batch_set_plan(ctx, b, bplan)
            assert nb.nbody_batch_get_plan(ctx, b) == bplan
        allsys = nb.System.from_arrays(packed)
        nb.nbody_accel_batched(ctx, b, allsys)
        torch.cuda.synchronize()
        got = allsys.numpy()
        for k, (sp, ic, prm) in enumerate(zip(SPECS, parts, prms)):
            lo, hi = off[k], off[k + 1]
            plan = nb.nbody_batch_system_plan(ctx, b, k)
            if bplan is not None and sp[1] > 256 * 2 * max(bplan["split"], 1) and sp[4] != "fp32":
                assert bplan["split"] == 0 or plan["split"] > 1, (k, plan)
            alone = single(nb, ctx, ic, prm, plan, lambda s: nb.nbody_accel(ctx, s, prm))
            for key in ("ax", "ay", "az"):
                assert np.array_equal(got[key][lo:hi], alone[key]), (k, key, plan)
            if sp[1] >= 2:
                ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, sp[3], want_scale=True)
                if sp[5]:
                    h = wl.default_halo()
                    hx, hy, hz = orc.halo_accel(ic["x"], ic["y"], ic["z"], orc.Halo(h.v2, h.rc))
                    ax, ay, az = ax + hx, ay + hy, az + hz
                    A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
                e = force_errors(np.stack([got["ax"][lo:hi], got["ay"][lo:hi], got["az"][lo:hi]]),
                                 np.stack([ax, ay, az]), A)
                gate = {"fp64": 1e-12, "mixed": 2e-6, "fp32": 1e-3}[sp[4]]
                print(f"[err] batched {plan_id(bplan)} system {k} {sp[4]}: {e}", flush=True)
                assert e["eps_cond"] <= gate, (k, e)
                if sp[4] == "fp64":
                    assert e["eps_rms"] <= 1e-12, (k, e)
    finally:
        nb.nbody_batch_destroy(ctx, b)


@pytest.mark.parametrize("bplan", [None, BATCH_PLANS[2]], ids=plan_id)
@pytest.mark.parametrize("scheme", ["kdk", "o4"])
def test_steps_batched_equal_single(nb, ctx, scheme, bplan):
    packed, off, parts = make_batch(SPECS)
    prms = [params_of(nb, sp) for sp in SPECS]
    b = nb.nbody_batch_create(ctx, off, prms, [sp[6] for sp in SPECS])
    try:
        if bplan is not None:
            nb.nbody_batch_set_plan(ctx, b, bplan)
        allsys = nb.System.from_arrays(packed)
        nb.nbody_accel_batched(ctx, b, allsys)
        (nb.nbody_step_kdk_batched if scheme == "kdk" else nb.nbody_step_o4_batched)(ctx, b, allsys, 3)
        torch.cuda.synchronize()
        got = allsys.numpy()
        for k, (sp, ic, prm) in enumerate(zip(SPECS, parts, prms)):
            lo, hi = off[k], off[k + 1]
            step = nb.nbody_step_kdk if scheme == "kdk" else nb.nbody_step_o4

            def run(s, prm=prm, sp=sp, step=step):
                nb.nbody_accel(ctx, s, prm)
                step(ctx, s, prm, sp[6], 3)

            alone = single(nb, ctx, ic, prm, nb.nbody_batch_system_plan(ctx, b, k), run)
            for key in K:
                assert np.array_equal(got[key][lo:hi], alone[key]), (scheme, k, key)
    finally:
        nb.nbody_batch_destroy(ctx, b)


@pytest.mark.parametrize("scheme", ["kdk", "o4"])
def test_graph_replay_equals_eager(nb, ctx, scheme):
    packed, off, parts = make_batch(SPECS)
    prms = [params_of(nb, sp) for sp in SPECS]
    dts = [sp[6] for sp in SPECS]
    be = nb.nbody_batch_create(ctx, off, prms, dts)
    bg = nb.nbody_batch_create(ctx, off, prms, dts, flags=nb.NB_BATCH_GRAPH)
    step = nb.nbody_step_kdk_batched if scheme == "kdk" else nb.nbody_step_o4_batched
    try:
        se = nb.System.from_arrays(packed)
        sg = nb.System.from_arrays(packed)
        nb.nbody_accel_batched(ctx, be, se)
        nb.nbody_accel_batched(ctx, bg, sg)
        for rep in range(4):
            step(ctx, be, se, 2)
            step(ctx, bg, sg, 2)  # first call captures, later calls replay
            # eager work and a synchronisation between replays
            junk = torch.randn(1000, device="cuda").sum()
            torch.cuda.synchronize()
            for key in K:
                assert torch.equal(se[key], sg[key]), (scheme, rep, key)
        del junk
    finally:
        nb.nbody_batch_destroy(ctx, be)
        nb.nbody_batch_destroy(ctx, bg)


def test_isolation_and_order(nb, ctx):
    # reversing the order of systems in the pack changes no system's result
    packed, off, parts = make_batch(SPECS)
    prms = [params_of(nb, sp) for sp in SPECS]
    rs = SPECS[::-1]
    rpacked, roff, _ = make_batch(rs)
    b1 = nb.nbody_batch_create(ctx, off, prms, [sp[6] for sp in SPECS])
    b2 = nb.nbody_batch_create(ctx, roff, prms[::-1], [sp[6] for sp in rs])
    try:
        s1, s2 = nb.System.from_arrays(packed), nb.System.from_arrays(rpacked)
        for b, s in ((b1, s1), (b2, s2)):
            nb.nbody_accel_batched(ctx, b, s)
            nb.nbody_step_kdk_batched(ctx, b, s, 2)
        torch.cuda.synchronize()
        g1, g2 = s1.numpy(), s2.numpy()
        B = len(SPECS)
        for k in range(B):
            r = B - 1 - k
            for key in K:
                assert np.array_equal(g1[key][off[k]:off[k + 1]], g2[key][roff[r]:roff[r + 1]])
    finally:
        nb.nbody_batch_destroy(ctx, b1)
        nb.nbody_batch_destroy(ctx, b2)


LARGE_SPECS = [
    ("disk", 40000, 21, 0.02, "mixed", True, 1e-3),
    ("plummer", 700, 22, 0.01, "mixed", False, 1e-3),
    ("plummer", 33000, 23, 0.01, "mixed", False, 2e-3),
    ("disk", 5000, 24, 0.02, "fp64", True, 1e-3),
    ("plummer", 0, 25, 0.01, "mixed", False, 1e-3),
    ("disk", 32768, 26, 0.02, "mixed", True, 1e-3),
    ("plummer", 9000, 27, 0.01, "mixed", False, 1e-3),
]


@pytest.mark.parametrize("bplan", [{"R": 1, "block": 256, "split": 16, "jsrc": 3},
                                   {"R": 2, "block": 256, "split": 0, "jsrc": 2},
                                   {"R": 1, "block": 256, "split": 7, "jsrc": 2},
                                   {"R": 2, "block": 256, "split": 16, "jsrc": 4},
                                   {"R": 1, "block": 256, "split": 0, "jsrc": 4},
                                   {"R": 2, "block": 256, "split": 8, "jsrc": 5}], ids=plan_id)
def test_spatial_order_batch_large_systems(nb, ctx, orc, bplan):
    # mixed systems of 2^15 particles or more (2^12 under the quarter-tile
    # form) are summed in their own spatial order inside the batch (the
    # smaller ones with LDS tiles): bitwise the
    # single-system sums under the reported plans, and the oracle's on
    # sampled rows; one graph-replayed KDK step equals the eager one
    print(f"[case] batched large systems plan {bplan}", flush=True)
    packed, off, parts = make_batch(LARGE_SPECS)
    prms = [params_of(nb, sp) for sp in LARGE_SPECS]
    dts = [sp[6] for sp in LARGE_SPECS]
    b = nb.nbody_batch_create(ctx, off, prms, dts, flags=nb.NB_BATCH_GRAPH)
    try:
        nb.nbody_batch_set_plan(ctx, b, bplan)
        allsys = nb.System.from_arrays(packed)
        nb.nbody_accel_batched(ctx, b, allsys)
        torch.cuda.synchronize()
        got = allsys.numpy()
        rng = np.random.default_rng(9)
        for k, (sp, ic, prm) in enumerate(zip(LARGE_SPECS, parts, prms)):
            lo, hi = off[k], off[k + 1]
            plan = nb.nbody_batch_system_plan(ctx, b, k)
            # spatial order from 2^15 particles on (2^12 for the quarter-tile forms)
            if sp[4] == "mixed" and sp[1] >= (1 << 12 if bplan["jsrc"] >= 4 else 1 << 15):
                assert plan["jsrc"] == bplan["jsrc"], (k, plan)
            elif sp[1] > 0:
                assert plan["jsrc"] == 0, (k, plan)
            alone = single(nb, ctx, ic, prm, plan, lambda s, prm=prm: nb.nbody_accel(ctx, s, prm))
            for key in ("ax", "ay", "az"):
                assert np.array_equal(got[key][lo:hi], alone[key]), (k, key, plan)
            if sp[1] < 2:
                continue
            rows = np.sort(rng.choice(sp[1], size=min(256, sp[1]), replace=False))
            ax, ay, az, A = orc.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, sp[3], rows=rows, want_scale=True)
            if sp[5]:
                h = wl.default_halo()
                hx, hy, hz = orc.halo_accel(ic["x"][rows], ic["y"][rows], ic["z"][rows], orc.Halo(h.v2, h.rc))
                ax, ay, az = ax + hx, ay + hy, az + hz
                A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
            e = force_errors(np.stack([got["ax"][lo:hi][rows], got["ay"][lo:hi][rows], got["az"][lo:hi][rows]]),
                             np.stack([ax, ay, az]), A)
            print(f"[err] batched large {plan_id(bplan)} system {k}: {e}", flush=True)
            gate = {"fp64": 1e-12, "mixed": 2e-6}[sp[4]]
            assert e["eps_cond"] <= gate and e["eps_rms"] <= gate, (k, e)
        # graph replay of a step equals the eager step
        eager = nb.System.from_arrays(got)
        be = nb.nbody_batch_create(ctx, off, prms, dts)
        try:
            nb.nbody_batch_set_plan(ctx, be, bplan)
            for _ in range(2):
                nb.nbody_step_kdk_batched(ctx, b, allsys, 1)
                nb.nbody_step_kdk_batched(ctx, be, eager, 1)
                torch.cuda.synchronize()
                for key in K:
                    assert torch.equal(allsys[key], eager[key]), key
        finally:
            nb.nbody_batch_destroy(ctx, be)
    finally:
        nb.nbody_batch_destroy(ctx, b)


def test_batch_reset_reuses_and_matches_create(nb, ctx):
    # a batch reset for another set of systems gives the bits of a batch
    # created for that set, on the stream the reset was ordered on
    specs_a, specs_b = SPECS, LARGE_SPECS
    pa, offa, _ = make_batch(specs_a)
    pb, offb, _ = make_batch(specs_b)
    prm_a = [params_of(nb, sp) for sp in specs_a]
    prm_b = [params_of(nb, sp) for sp in specs_b]
    st = torch.cuda.Stream()
    b = nb.nbody_batch_create(ctx, offa, prm_a, [sp[6] for sp in specs_a], flags=nb.NB_BATCH_GRAPH)
    ref = nb.nbody_batch_create(ctx, offb, prm_b, [sp[6] for sp in specs_b])
    try:
        sa = nb.System.from_arrays(pa)
        with torch.cuda.stream(st):
            nb.nbody_accel_batched(ctx, b, sa, stream=st)
            nb.nbody_step_kdk_batched(ctx, b, sa, 2, stream=st)
            nb.nbody_batch_reset(ctx, b, offb, prm_b, [sp[6] for sp in specs_b], stream=st)
            s1 = nb.System.from_arrays(pb)
            nb.nbody_accel_batched(ctx, b, s1, stream=st)
            nb.nbody_step_kdk_batched(ctx, b, s1, 3, stream=st)
        st.synchronize()
        assert nb.nbody_batch_get_plan(ctx, b) == nb.nbody_batch_get_plan(ctx, ref)
        s2 = nb.System.from_arrays(pb)
        nb.nbody_accel_batched(ctx, ref, s2)
        nb.nbody_step_kdk_batched(ctx, ref, s2, 3)
        torch.cuda.synchronize()
        for key in K:
            assert torch.equal(s1[key], s2[key]), key
        with pytest.raises(nb.NBodyError):
            nb.nbody_batch_reset(ctx, b, [0, 5, 3], prm_b[:2])
    finally:
        nb.nbody_batch_destroy(ctx, b)
        nb.nbody_batch_destroy(ctx, ref)


def test_diag_batched(nb, ctx, orc):
    packed, off, parts = make_batch(SPECS)
    prms = [params_of(nb, sp) for sp in SPECS]
    b = nb.nbody_batch_create(ctx, off, prms)
    try:
        s = nb.System.from_arrays(packed)
        out = nb.nbody_diag_batched(ctx, b, s, len(SPECS)).cpu().numpy()
        for k, (sp, ic) in enumerate(zip(SPECS, parts)):
            if sp[1] == 0:
                assert np.all(out[k] == 0)
                continue
            h = wl.default_halo()
            r = orc.diag(ic, 1.0, sp[3], orc.Halo(h.v2, h.rc) if sp[5] else None)
            g = dict(zip(nb.DIAG_KEYS, out[k].tolist()))
            for key in ("K", "W", "Wext", "E", "M"):
                assert abs(g[key] - r[key]) <= 1e-12 * max(abs(r[key]), 1e-300), (k, key, g[key], r[key])
            for key in ("Px", "Py", "Pz", "Lx", "Ly", "Lz"):
                assert abs(g[key] - r[key]) <= 1e-14, (k, key)
    finally:
        nb.nbody_batch_destroy(ctx, b)


def test_batch_validation(nb, ctx):
    p = nb.Params(eps=0.01)
    with pytest.raises(nb.NBodyError):
        nb.nbody_batch_create(ctx, [0, 5, 3], [p, p])       # non-monotone offsets
    with pytest.raises(nb.NBodyError):
        nb.nbody_batch_create(ctx, [1, 5], [p])             # off[0] != 0
    with pytest.raises(nb.NBodyError):
        nb.nbody_batch_create(ctx, [0, 5], [nb.Params(eps=-1.0)])
    with pytest.raises(nb.NBodyError):
        nb.nbody_batch_create(ctx, [0, 5], [p], [float("inf")])
    b = nb.nbody_batch_create(ctx, [0, 5, 9], [p, p], [1e-3, 1e-3])
    try:
        with pytest.raises(nb.NBodyError):                   # all.n != off[B]
            nb.nbody_accel_batched(ctx, b, nb.System(8))
    finally:
        nb.nbody_batch_destroy(ctx, b)


def test_batch_mix_full_size_sampled(nb, ctx, orc):
    # 256 systems, N log-uniform in [2^10, 2^16] (half Plummer, half disk),
    # mixed precision as in the batched workload; 32 sampled rows per system
    print("[case] batch mix 256 systems, mixed", flush=True)
    mix = wl.batch_mix(256, 4)
    off = mix["off"]
    B = len(off) - 1
    h = wl.default_halo()
    prms = [nb.Params(eps=0.01 if mix["kind"][k] == "plummer" else 0.02, prec=nb.NB_MIXED,
                      halo=mix["kind"][k] == "disk", halo_v2=h.v2, halo_rc=h.rc) for k in range(B)]
    b = nb.nbody_batch_create(ctx, off, prms, [1e-3] * B, flags=nb.NB_BATCH_GRAPH)
    try:
        s = nb.System.from_arrays(mix)
        nb.nbody_accel_batched(ctx, b, s)
        torch.cuda.synchronize()
        got = s.numpy()
        rng = np.random.default_rng(3)
        worst = 0.0
        for k in range(B):
            lo, hi = int(off[k]), int(off[k + 1])
            rows = np.sort(rng.choice(hi - lo, size=32, replace=False))
            sl = {f: mix[f][lo:hi] for f in ("x", "y", "z", "m")}
            ax, ay, az, A = orc.accel(sl["x"], sl["y"], sl["z"], sl["m"], 1.0, prms[k].eps, rows=rows,
                                      want_scale=True)
            if prms[k].halo:
                hx, hy, hz = orc.halo_accel(sl["x"][rows], sl["y"][rows], sl["z"][rows], orc.Halo(h.v2, h.rc))
                ax, ay, az = ax + hx, ay + hy, az + hz
                A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
            e = force_errors(np.stack([got["ax"][lo:hi][rows], got["ay"][lo:hi][rows], got["az"][lo:hi][rows]]),
                             np.stack([ax, ay, az]), A)
            worst = max(worst, e["eps_cond"])
        print(f"[err] batched mix worst eps_cond {worst:.3e}", flush=True)
        assert worst <= 2e-6, worst   # measured 6.5e-7
        # the largest, the smallest and two other systems alone, under the
        # plan the batch reports for each: bitwise the batch's sums
        sizes = np.diff(off)
        for k in (int(np.argmax(sizes)), int(np.argmin(sizes)), 17, 200):
            lo, hi = int(off[k]), int(off[k + 1])
            ic = {f: mix[f][lo:hi] for f in wl.FIELDS}
            alone = single(nb, ctx, ic, prms[k], nb.nbody_batch_system_plan(ctx, b, k),
                           lambda s, k=k: nb.nbody_accel(ctx, s, prms[k]))
            for key in ("ax", "ay", "az"):
                assert np.array_equal(got[key][lo:hi], alone[key]), (k, key)
    finally:
        nb.nbody_batch_destroy(ctx, b)
