"""The spatial (Morton) order behind the jsrc 2 to 5 plans is computed by
the library's own kernels (bounding box, keys, an eight-pass stable radix
sort, gathers).  Its permutation must be exactly the stable sort of the keys
that nbody_spatial_order's contract defines, recomputed here on the host; and
because the ordering has no library sort, memset or host synchronisation, a
step under a spatially ordered plan can be captured into a HIP graph and
replays bit for bit like the eager call."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def host_keys(x, y, z):
    """Morton keys as the header defines them, in numpy float64 / uint64."""
    p = [np.asarray(c, dtype=np.float64) for c in (x, y, z)]
    lo = [np.min(c) for c in p]
    hi = [np.max(c) for c in p]
    ext = max(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
    s = 2097151.0 / ext if ext > 0 else 0.0
    key = np.zeros(p[0].size, dtype=np.uint64)
    for c in range(3):
        q = (p[c] - lo[c]) * s
        q = np.fmin(np.fmax(q, 0.0), 2097151.0)
        q = np.nan_to_num(q, nan=0.0).astype(np.uint64)
        for b in range(21):
            key |= ((q >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + c)
    return key


CASES = {
    "plummer_1": lambda: wl.plummer(1, 1),
    "plummer_255": lambda: wl.plummer(255, 2),
    "plummer_257": lambda: wl.plummer(257, 3),
    "disk_5000": lambda: wl.exp_disk(5000, 4),
    "plummer_70001": lambda: wl.plummer(70001, 5),
    "disk_300001": lambda: wl.exp_disk(300001, 6),   # 586 sort blocks of 2 tiles
    "disk_2p20": lambda: wl.exp_disk(1 << 20, 2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_permutation_is_stable_sort_of_keys(nb, ctx, case):
    print(f"[case] spatial order {case}", flush=True)
    ic = CASES[case]()
    n = len(ic["x"])
    if case == "disk_5000":
        # ties: coincident particles and a flat coordinate
        ic = {k: v.copy() for k, v in ic.items()}
        ic["x"][100:400] = ic["x"][7]
        ic["y"][100:400] = ic["y"][7]
        ic["z"][100:400] = ic["z"][7]
    s = nb.System.from_arrays(ic)
    perm, keys = nb.nbody_spatial_order(ctx, s)
    torch.cuda.synchronize()
    want_keys = host_keys(ic["x"], ic["y"], ic["z"])
    want = np.argsort(want_keys, kind="stable")
    got = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(got), np.arange(n))
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), want_keys[want])
    assert np.array_equal(got, want)


def test_flat_system_and_zero_extent(nb, ctx):
    # every particle at one point: extent 0, all keys 0, identity order
    n = 1000
    ic = {k: np.zeros(n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    ic["m"] = np.full(n, 1.0 / n)
    s = nb.System.from_arrays(ic)
    perm, keys = nb.nbody_spatial_order(ctx, s)
    assert np.array_equal(perm.cpu().numpy(), np.arange(n))
    assert not keys.cpu().numpy().any()


@pytest.mark.parametrize("kind", ["accel", "jerk"])
def test_spatial_plan_graph_capture_matches_eager(nb, ctx, kind):
    # the tuned mixed plans at N = 2^17 (spatial order, split sums):
    # KDK (or Hermite) steps captured in a graph replay bitwise like eager calls
    n = 1 << 17
    print(f"[case] graph capture spatial plan {kind} n={n}", flush=True)
    nb.load_plans(ctx)
    code = nb.NB_MIXED | (nb.NB_PLAN_JERK if kind == "jerk" else 0)
    assert nb.nbody_plan_get(ctx, code, n)["jsrc"] >= 2
    ic = wl.exp_disk(n, 21)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    init = nb.nbody_accel_jerk if kind == "jerk" else nb.nbody_accel
    step = nb.nbody_step_hermite if kind == "jerk" else nb.nbody_step_kdk
    eager = nb.System.from_arrays(ic)
    cap = nb.System.from_arrays(ic)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for sy in (eager, cap):
            init(ctx, sy, prm, stream=st)
        step(ctx, cap, prm, 1e-3, 1, stream=st)     # warm-up sizes the scratch
        step(ctx, eager, prm, 1e-3, 1, stream=st)
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        step(ctx, cap, prm, 1e-3, 2, stream=st)
    keys = ("x", "vx", "ax", "az") + (("jx",) if kind == "jerk" else ())
    for rep in range(3):
        g.replay()
        step(ctx, eager, prm, 1e-3, 2)
        junk = torch.randn(4096, device="cuda").cumsum(0)  # unrelated eager work
        torch.cuda.synchronize()
        for k in keys:
            a = eager.jerk(k) if k.startswith("j") else eager[k]
            b = cap.jerk(k) if k.startswith("j") else cap[k]
            assert torch.equal(a, b), (kind, rep, k)
    del junk


def test_capture_refuses_to_grow_scratch(nb, ctx):
    # a spatially ordered call whose scratch is too small under capture
    # fails with NB_EINVAL instead of allocating inside the capture
    n = 3 * (1 << 21)   # larger than anything sized before in this session
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, {"R": 1, "block": 256, "split": 1, "jsrc": 3})
    try:
        ic = {k: np.linspace(0.0, 1.0, n) for k in ("x", "y", "z")}
        ic["m"] = np.full(n, 1.0 / n)
        s = nb.System.from_arrays(ic)
        st = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with pytest.raises(nb.NBodyError) as ei:
            with torch.cuda.graph(g, stream=st):
                nb.nbody_accel(ctx, s, nb.Params(eps=0.02, prec=nb.NB_MIXED), stream=st)
        assert ei.value.status == nb.NB_EINVAL and "capture" in str(ei.value)
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)


@pytest.mark.parametrize("plan", [{"R": 1, "block": 256, "split": 4, "jsrc": 3},
                                  {"R": 2, "block": 256, "split": 1, "jsrc": 2},
                                  {"R": 2, "block": 256, "split": 3, "jsrc": 4},
                                  {"R": 1, "block": 256, "split": 2, "jsrc": 5}], ids=["R1s4j3", "R2s1j2", "R2s3j4", "R1s2j5"])
def test_order_rows_bitwise(nb, ctx, plan):
    # the i-split under a spatially ordered plan: ranges of the Morton order
    # give the full launch's bits for their particles and touch no others;
    # three ranges cover the system exactly
    n = 40000
    print(f"[case] order rows n={n} plan={plan}", flush=True)
    ic = wl.exp_disk(n, 23)
    h = wl.default_halo()
    prm = nb.Params(eps=0.02, prec=nb.NB_MIXED, halo=True, halo_v2=h.v2, halo_rc=h.rc)
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, plan)
    try:
        full = nb.System.from_arrays(ic)
        nb.nbody_accel(ctx, full, prm)
        perm, _ = nb.nbody_spatial_order(ctx, full)
        part = nb.System.from_arrays(ic)
        for k in ("ax", "ay", "az"):
            part[k].fill_(7.0)
        k0, k1 = 1000, 23456
        nb.nbody_accel_order_rows(ctx, part, prm, k0, k1)
        torch.cuda.synchronize()
        p = perm.long()
        inside = torch.zeros(n, dtype=torch.bool, device="cuda")
        inside[p[k0:k1]] = True
        for k in ("ax", "ay", "az"):
            assert torch.equal(part[k][inside], full[k][inside]), k
            assert torch.all(part[k][~inside] == 7.0), k
        whole = nb.System.from_arrays(ic)
        for a, b in ((0, 777), (777, 31000), (31000, n)):
            nb.nbody_accel_order_rows(ctx, whole, prm, a, b)
        torch.cuda.synchronize()
        for k in ("ax", "ay", "az"):
            assert torch.equal(whole[k], full[k]), k
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_accel_order_rows(ctx, whole, prm, 5, n + 1)
        assert ei.value.status == nb.NB_EINVAL
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)
    # a plan that is not spatially ordered has no such order
    nb.nbody_plan_set(ctx, nb.NB_MIXED, n, {"R": 1, "block": 256, "split": 1, "jsrc": 0})
    try:
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_accel_order_rows(ctx, nb.System.from_arrays(ic), prm, 0, 10)
        assert ei.value.status == nb.NB_ENOTSUP
    finally:
        nb.nbody_plan_set(ctx, nb.NB_MIXED, n, None)
