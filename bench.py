"""Benchmark: pair-interactions/s of the direct-sum N-body step at N = 2^20.

Workload: gravitationally unstable exponential stellar disk, N = 2^20
(surface density ~ exp(-R/h), h = 1, cut at R = 4h, sech^2(z/z0) with
z0 = 0.1, disk mass 1, fixed cored isothermal halo, Toomre Q = 1.2),
softening eps = 0.02, leapfrog KDK dt = 1e-3.  A step is one KDK step:
kick-drift, the O(N^2) pair sum with the halo field and the closing kick.
The headline value is the mixed-precision path; float64 and float32 are
timed the same way and reported alongside.  Inputs are resident in HBM
before the timed region starts.

Prints ONE JSON line (see the keys below).  --gpus above 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

T_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s at N=2^20 (FP64 vs mixed @ stated err); p50/p99 latency"
FLOPS_PER_INTERACTION = 20  # conventional count for the softened pair term
JERK_FLOPS_PER_INTERACTION = 42  # the 20 above + relative velocity (3), r.u (5), factor (2), jerk FMAs (12)
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3, "fp32": 157.3}  # MI355X vector peaks
# VALU issue quad-cycles per lane-interaction of each precision's tuned pair
# kernel after dual issue (SQ counters on the N = 2^20 disk,
# profiles/pmc_valu_disk_2p20.md); 1024 SIMDs each issue one wave64
# instruction per quad-cycle, so the issue-limited rate is 16384 f / qc at
# clock f (the 2.4 GHz peak clock is used).
ISSUE_QC = {"fp64": 18.07, "mixed": 9.57, "fp32": 10.28}
PEAK_CLOCK_HZ = 2.4e9
MIN_LATENCY_SAMPLES = 50
DTYPE = {"fp64": "f64", "mixed": "f32 pair / f64 accumulate+state", "fp32": "f32"}
KERNEL_SOURCES = ["paper_1803_01190_amd/csrc/accel.hip", "paper_1803_01190_amd/csrc/order.hip",
                  "paper_1803_01190_amd/csrc/halo.h",
                  "paper_1803_01190_amd/csrc/nbody_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(prec: str, plan: dict = None):
    """HBM bytes per pair-sum launch from the committed rocprofv3 counter
    summary, or None when the kernel source or the launch plan changed since
    it was taken (the split partial sums are part of the traffic)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    if plan is not None and rec.get("plans", {}).get(prec) != plan:
        return None
    return rec.get("per_launch_bytes", {}).get(prec)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--precs", default="mixed,fp64,fp32")
    ap.add_argument("--tune-ms", type=float, default=4000.0)
    ap.add_argument("--sample-rows", type=int, default=32768,
                    help="oracle rows (each summed over all N) for the CPU baseline and force errors")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plans-in", default=None,
                    help="plan-cache JSON ({arch: {prec: {log2n: plan}}}); default: the committed "
                         "tuned_plans.json when it has this size, else autotune")
    ap.add_argument("--retune", action="store_true", help="autotune even if a cached plan exists")
    ap.add_argument("--plans-out", default=None, help="write the plans used in plan-cache form")
    ap.add_argument("--workload", default="disk",
                    choices=["disk", "batched", "serving", "integrators", "longrun", "hermite", "scaling"],
                    help="disk: the headline N=2^20 step (default); batched: 256 independent systems "
                         "in one persistent launch vs one launch per system; serving: Poisson "
                         "request stream through the continuous-batching loop; longrun: 10^4-step "
                         "self-gravitating disk in each precision (conservation and density maps); "
                         "hermite: the fourth-order Hermite step at N=2^20; scaling: one step for "
                         "N = 2^17..2^23 (Table 1)")
    ap.add_argument("--long-n", type=int, default=1 << 17, help="longrun: particles")
    ap.add_argument("--long-steps", type=int, default=10000, help="longrun: steps per run")
    ap.add_argument("--long-runs", default="fp64,fp64_alt,mixed,fp32",
                    help="longrun: runs (fp64_alt: float64 with another summation order)")
    ap.add_argument("--out-dir", default="longrun_out", help="longrun: series and maps")
    ap.add_argument("--long-equilibrium", action="store_true",
                    help="longrun: start from the disk iterated to equilibrium (Eqs. (3)-(4))")
    ap.add_argument("--stop-at", type=int, default=None,
                    help="longrun: stop each run at this step and save it for --resume-dir")
    ap.add_argument("--resume-dir", default=None, help="longrun: continue the runs saved there")
    ap.add_argument("--stop-after-s", type=float, default=None,
                    help="longrun: stop each run at its first sample point after this many seconds "
                         "(from the start of the program) and save it for --resume-dir")
    ap.add_argument("--scaling-max-log2", type=int, default=23, help="scaling: largest N = 2^k")
    ap.add_argument("--requests", type=int, default=12, help="serving: requests per arrival rate")
    ap.add_argument("--no-graph", action="store_true", help="serving: launch every step (no HIP graph replay)")
    ap.add_argument("--serve-log2", default="12-20", help="serving: request sizes N = 2^lo .. 2^hi (log-uniform)")
    ap.add_argument("--serve-steps", default="10-1000", help="serving: steps per request (uniform)")
    ap.add_argument("--rates", default="0.5,0.9,1.1", help="serving: arrival rates as fractions of capacity")
    ap.add_argument("--capacity", type=float, default=None,
                    help="serving: capacity in requests/s (skip its measurement)")
    ap.add_argument("--serve-out", default=None, help="serving: also write the result JSON here")
    ap.add_argument("--integ-out", default=None, help="integrators: also write the result JSON here")
    ap.add_argument("--batch-tune-ms", type=float, default=3000.0,
                    help="batched: autotune the batch plan on the batch first (0: the pinned or default plan)")
    ap.add_argument("--profile-run", action="store_true",
                    help="run for counter collection: no CPU baseline, plus a copy kernel of "
                         "known size to calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(splitting the targets across GPUs is designed but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "integrators":
        return bench_integrators(args)
    if args.workload == "longrun":
        return bench_longrun(args)
    if args.workload == "hermite":
        return bench_hermite(args)
    if args.workload == "scaling":
        return bench_scaling(args)
    dev = torch.device("cuda:0")
    n, dt, eps = args.n, 1e-3, 0.02
    halo = wl.default_halo()
    t_ic = time.perf_counter()
    ic = wl.exp_disk(n, 2)
    log(f"[bench] disk N={n} generated in {time.perf_counter() - t_ic:.1f}s")
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]

    ctx = nb.Context(0)
    base = nb.System.from_arrays(ic, device=dev)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n, size=min(args.sample_rows, n), replace=False))
    rows_t = torch.as_tensor(rows, device=dev)

    log2n = max(0, (n - 1).bit_length())
    pinned = {}
    if not args.retune:
        table = nb.read_plans(args.plans_in) if args.plans_in else nb.read_plans()
        pinned = {k: v[str(log2n)] for k, v in table.items() if str(log2n) in v}
        for k, v in pinned.items():  # potential-pass and jerk plans of this size
            if "/" in k:
                nb.nbody_plan_set(ctx.h, nb.plan_code(k), n, v)
    results = {}
    for prec in precs:
        p = nb.PREC[prec]
        prm = nb.Params(G=1.0, eps=eps, prec=p, halo=True, halo_v2=halo.v2, halo_rc=halo.rc)
        t0 = time.perf_counter()
        if prec in pinned:
            nb.nbody_plan_set(ctx.h, p, n, pinned[prec])
            plan = nb.nbody_plan_get(ctx.h, p, n)
        elif args.tune_ms > 0:
            plan = nb.nbody_autotune(ctx.h, p, n, args.tune_ms)
        else:
            plan = nb.nbody_plan_get(ctx.h, p, n)
        log(f"[bench] {prec}: plan {plan} ({time.perf_counter() - t0:.1f}s)")
        s = nb.System(n, device=dev)
        for k in nb.FIELDS:
            s.t[k].copy_(base.t[k])
        nb.nbody_accel(ctx.h, s, prm)
        a0 = torch.stack([s["ax"][rows_t], s["ay"][rows_t], s["az"][rows_t]]).cpu().numpy()
        for _ in range(args.warmup):
            nb.nbody_step_kdk(ctx.h, s, prm, dt, 1)
        d0 = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
        torch.cuda.synchronize()
        nb.nbody_profile_read(ctx.h)
        nb.nbody_profile_enable(ctx.h, True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            nb.nbody_step_kdk(ctx.h, s, prm, dt, 1)
            evs[k + 1].record()
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        nb.nbody_profile_enable(ctx.h, False)
        prof = nb.nbody_profile_read(ctx.h)
        d1 = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
        step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        if prec == precs[0] and args.steps < MIN_LATENCY_SAMPLES and not args.profile_run:
            # more per-step latency samples for p50/p99, after the timed region
            extra = MIN_LATENCY_SAMPLES - args.steps
            ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(extra + 1)]
            ev2[0].record()
            for k in range(extra):
                nb.nbody_step_kdk(ctx.h, s, prm, dt, 1)
                ev2[k + 1].record()
            torch.cuda.synchronize()
            step_ms += [ev2[k].elapsed_time(ev2[k + 1]) for k in range(extra)]
        wall = w1 - w0
        inter = float(n) * float(n)
        rate = args.steps * inter / wall
        accel_ms = prof["accel_ms"] / max(prof["accel_launches"], 1)
        tflops = FLOPS_PER_INTERACTION * inter / (accel_ms * 1e-3) / 1e12
        m_tot = float(np.sum(ic["m"]))
        results[prec] = {
            "value": rate,
            "ms_per_step": 1e3 * wall / args.steps,
            "latency_ms": {"p50": percentile(step_ms, 0.5), "p99": percentile(step_ms, 0.99),
                           "samples": len(step_ms)},
            "plan": plan,
            "accel_kernel_ms": accel_ms,
            "accel_launches": prof["accel_launches"],
            "update_ms_per_step": prof["update_ms"] / max(args.steps, 1),
            "achieved_tflops": tflops,
            "drift": {
                "dE_rel": abs(d1["E"] - d0["E"]) / abs(d0["E"]),
                "dLz_rel": abs(d1["Lz"] - d0["Lz"]) / abs(d0["Lz"]),
                "dP_abs": math.sqrt(sum((d1[k] - d0[k]) ** 2 for k in ("Px", "Py", "Pz"))),
                "steps": args.steps,
            },
            "_a0": a0,
        }
        log(f"[bench] {prec}: {rate:.4e} pair-int/s, {1e3 * wall / args.steps:.1f} ms/step, "
            f"pair kernel {accel_ms:.1f} ms ({tflops:.1f} TFLOP/s at {FLOPS_PER_INTERACTION} flop/pair)")
        del s
        torch.cuda.empty_cache()

    if args.profile_run:
        # calibration copy of known size for the HBM byte counters
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 3 x 256 MiB")

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ----
    cpu = None
    force_err = {}
    if not args.no_cpu_baseline and not args.profile_run:
        import oracle
        from oracle.metrics import force_errors
        oracle.build(force=False)
        cores = oracle.max_threads()
        t0 = time.perf_counter()
        ax, ay, az, A = oracle.accel(ic["x"], ic["y"], ic["z"], ic["m"], 1.0, eps, rows=rows, want_scale=True)
        el = time.perf_counter() - t0
        hx, hy, hz = oracle.halo_accel(ic["x"][rows], ic["y"][rows], ic["z"][rows], oracle.Halo(halo.v2, halo.rc))
        ref = np.stack([ax + hx, ay + hy, az + hz])
        A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
        cpu = {"value": rows.size * float(n) / el, "unit": "pair-interactions/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{rows.size} seeded rows of the N=2^20 disk, each summed over all {n} sources "
                         f"(float64 direct sum, {el:.1f} s on {cores} threads)"}
        for prec, r in results.items():
            force_err[prec] = force_errors(r["_a0"], ref, A)
        log(f"[bench] cpu oracle: {cpu['value']:.3e} pair-int/s on {cores} threads; errors {force_err}")

    if args.plans_out:
        with open(args.plans_out, "w") as f:
            json.dump({"gfx950": {k: {str(log2n): v["plan"]} for k, v in results.items()}}, f, indent=1)
    head = precs[0]
    r0 = results[head]
    traffic = load_traffic(head, r0["plan"])
    out = {
        "metric": METRIC,
        "value": r0["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r0["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"exponential stellar disk N={n} + fixed isothermal halo, eps={eps}, "
                               f"KDK dt={dt}", "n": n, "eps": eps, "dt": dt, "integrator": "kdk",
                   "precision": head, "seed": 2},
        "latency_ms": r0["latency_ms"],
        "roofline": {
            "bound": "alu",
            "achieved": r0["achieved_tflops"],
            "peak": PEAK_TFLOPS[head],
            "unit": "TFLOP/s",
            "frac": r0["achieved_tflops"] / PEAK_TFLOPS[head],
            "traffic": traffic,
            "kernel": ("pair sum in spatial order (k_pair_local, with its ordering kernels)"
                       if r0["plan"].get("jsrc") in (2, 3) else "pair sum (k_pair)"),
            "flops_per_interaction": FLOPS_PER_INTERACTION,
            "interactions_per_launch": float(n) * float(n),
        },
        # the binding limit of this VALU-bound kernel: its instruction issue
        "issue_roofline": {
            "bound": "valu issue",
            "unit": "pair-interactions/s",
            "achieved": float(n) * float(n) / (r0["accel_kernel_ms"] * 1e-3),
            "peak": 16384.0 * PEAK_CLOCK_HZ / ISSUE_QC[head],
            "frac": float(n) * float(n) / (r0["accel_kernel_ms"] * 1e-3) / (16384.0 * PEAK_CLOCK_HZ / ISSUE_QC[head]),
            "quad_cycles_per_interaction": ISSUE_QC[head],
            "clock_hz": PEAK_CLOCK_HZ,
            "source": "SQ_ACTIVE_INST_VALU / SQ_ACTIVE_INST_VALU2 counts of the pair kernel, "
                      "profiles/pmc_valu_disk_2p20.md",
        },
        "cpu_baseline": cpu,
        "force_error": force_err or None,
        "per_precision": {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")}
                          for k, v in results.items()},
    }
    print(json.dumps(out))
    ctx.close()


def bench_batched(args):
    """256 independent systems (half Plummer, half disk), N log-uniform in
    [2^10, 2^16], mixed precision, KDK: one persistent launch per step replayed
    from a HIP graph, against one launch per system per step."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    B, steps = 256, args.steps if args.steps != 10 else 100
    mix = wl.batch_mix(B, 4)
    off = mix["off"]
    sizes = np.diff(off)
    inter = float(np.sum(sizes.astype(np.float64) ** 2))
    h = wl.default_halo()
    prms = [nb.Params(eps=0.01 if mix["kind"][k] == "plummer" else 0.02, prec=nb.NB_MIXED,
                      halo=mix["kind"][k] == "disk", halo_v2=h.v2, halo_rc=h.rc) for k in range(B)]
    ctx = nb.Context(0)
    nb.load_plans(ctx.h)
    if args.plans_in:
        nb.load_plans(ctx.h, args.plans_in)
    out = {}
    # persistent + graph
    b = nb.nbody_batch_create(ctx.h, off, prms, [1e-3] * B, flags=nb.NB_BATCH_GRAPH)
    s = nb.System.from_arrays(mix)
    if args.batch_tune_ms > 0:
        t0 = time.perf_counter()
        plan = nb.nbody_batch_autotune(ctx.h, b, s, args.batch_tune_ms)
        log(f"[bench] batch plan tuned: {plan} ({time.perf_counter() - t0:.1f}s)")
    plan = nb.nbody_batch_get_plan(ctx.h, b)
    if args.plans_out:
        log2 = max(0, int(sizes.max() - 1).bit_length())
        with open(args.plans_out, "w") as f:
            json.dump({"gfx950": {"mixed/batch": {str(log2): plan}}}, f, indent=1)
    nb.nbody_accel_batched(ctx.h, b, s)
    nb.nbody_step_kdk_batched(ctx.h, b, s, 1)  # capture + warm-up
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    w0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        nb.nbody_step_kdk_batched(ctx.h, b, s, 1)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    lat = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    out["persistent_graph"] = {"value": steps * inter / wall, "ms_per_step": 1e3 * wall / steps,
                               "latency_ms": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99),
                                              "samples": len(lat)},
                               "plan": plan}
    sys_plans = [nb.nbody_batch_system_plan(ctx.h, b, k) for k in range(B)]
    nb.nbody_batch_destroy(ctx.h, b)
    log(f"[bench] batched persistent+graph: {out['persistent_graph']}")
    # one launch per system, each under the plan that gives the batch's bits
    # (so the two modes do the same arithmetic)
    systems = [nb.System.from_arrays({f: mix[f][off[k]:off[k + 1]] for f in wl.FIELDS}) for k in range(B)]

    def per_system_step(k):
        nb.nbody_plan_set(ctx.h, nb.NB_MIXED, int(sizes[k]), sys_plans[k])
        nb.nbody_step_kdk(ctx.h, systems[k], prms[k], 1e-3, 1)

    for k in range(B):
        nb.nbody_plan_set(ctx.h, nb.NB_MIXED, int(sizes[k]), sys_plans[k])
        nb.nbody_accel(ctx.h, systems[k], prms[k])
    ps = max(1, steps // 10)
    for k in range(B):
        per_system_step(k)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(ps):
        for k in range(B):
            per_system_step(k)
    torch.cuda.synchronize()
    wall1 = time.perf_counter() - w0
    out["one_launch_per_system"] = {"value": ps * inter / wall1, "ms_per_step": 1e3 * wall1 / ps, "steps": ps}
    log(f"[bench] one launch per system: {out['one_launch_per_system']}")
    res = {"metric": "batched pair-interactions/s (256 systems, N log-uniform 2^10..2^16, mixed)",
           "value": out["persistent_graph"]["value"], "unit": "pair-interactions/s", "n_gpus": 1,
           "steps": steps, "warmup": 1, "ms_per_step": out["persistent_graph"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE["mixed"],
           "data": "synthetic",
           "config": {"workload": "256 systems (128 Plummer, 128 disk), N_k log-uniform in [2^10, 2^16], "
                                  "seed 4, KDK dt=1e-3", "sum_n": int(off[-1]), "sum_n2": inter},
           "latency_ms": out["persistent_graph"]["latency_ms"], "modes": out,
           "speedup_vs_per_system": out["persistent_graph"]["value"] / out["one_launch_per_system"]["value"]}
    print(json.dumps(res))
    ctx.close()


def bench_integrators(args):
    """Second-order KDK vs the fourth-order schemes on the N = 2^17 disk
    (eps = 0.02, halo), in each precision, over T = 1: KDK, the triple-jump
    composition O4 and Hermite with dt = 1e-3 (1000 steps each), and
    cost-matched runs (O4 334 steps, RK4 250 steps: about 1000 force
    evaluations; Hermite 500 steps: its acceleration-and-jerk sum costs about
    two acceleration sums).  The long-run
    reference is the float64 O4 run at dt = 5e-4 on the GPU (its pair sum is
    the float64 path gated against the CPU oracle at 1e-12); the CPU oracle
    would need hours for these runs.  The CPU-baseline leg runs the oracle
    on 1024 sampled rows at every checkpoint of the reference run (each row
    summed over all N sources) and compares them with the reference's own
    float64 accelerations there (gate 1e-12, conditioned), which both times
    the oracle and pins the reference trajectory's forces."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    n, T = 1 << 17, 1.0
    ic = wl.exp_disk(n, 3)
    h = wl.default_halo()
    ctx = nb.Context(0)
    nb.load_plans(ctx.h)

    def params(prec):
        return nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)

    def run(prec, scheme, nsteps, every, check=None):
        prm = params(prec)
        s = nb.System.from_arrays(ic)
        nb.nbody_accel(ctx.h, s, prm)
        d0 = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
        worst = {"dE_rel": 0.0, "dLz_rel": 0.0, "dP_abs": 0.0}
        dt = T / nsteps
        step = {"kdk": nb.nbody_step_kdk, "o4": nb.nbody_step_o4, "hermite": nb.nbody_step_hermite,
                "rk4": nb.nbody_step_rk4}[scheme]
        if scheme == "hermite":
            nb.nbody_accel_jerk(ctx.h, s, prm)
        torch.cuda.synchronize()
        busy = 0.0
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            t0 = time.perf_counter()
            step(ctx.h, s, prm, dt, k)
            torch.cuda.synchronize()
            busy += time.perf_counter() - t0
            done += k
            if check is not None:
                check(done, s)
            d = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
            worst["dE_rel"] = max(worst["dE_rel"], abs(d["E"] - d0["E"]) / abs(d0["E"]))
            worst["dLz_rel"] = max(worst["dLz_rel"], abs(d["Lz"] - d0["Lz"]) / abs(d0["Lz"]))
            worst["dP_abs"] = max(worst["dP_abs"], math.sqrt(sum((d[c] - d0[c]) ** 2 for c in ("Px", "Py", "Pz"))))
        return s.numpy(), worst, busy

    # force error of each precision at t = 0 against float64
    f = {}
    for prec in ("fp64", "mixed", "fp32"):
        s = nb.System.from_arrays(ic)
        nb.nbody_accel(ctx.h, s, params(prec))
        f[prec] = np.stack([s["ax"].cpu().numpy(), s["ay"].cpu().numpy(), s["az"].cpu().numpy()])
    ref_a = f["fp64"]
    ferr = {p: float(np.sqrt(np.mean(((f[p] - ref_a) ** 2).sum(0) / (ref_a ** 2).sum(0)))) for p in ("mixed", "fp32")}
    log(f"[bench] rms relative force error vs fp64 at t=0: {ferr}")
    checks = []
    cpu = {"s": 0.0, "pairs": 0.0, "threads": None}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.metrics import force_errors

        rows = np.sort(np.random.default_rng(17).choice(n, size=1024, replace=False))
        halo = oracle.Halo(h.v2, h.rc)

        def check(step, s):
            # the oracle at the reference's current positions (1024 rows)
            st = {k: s[k].cpu().numpy() for k in ("x", "y", "z", "m", "ax", "ay", "az")}
            t0 = time.perf_counter()
            ax, ay, az, A = oracle.accel(st["x"], st["y"], st["z"], st["m"], 1.0, 0.02, rows=rows, want_scale=True)
            cpu["s"] += time.perf_counter() - t0
            cpu["pairs"] += float(rows.size) * n
            cpu["threads"] = oracle.max_threads()
            hx, hy, hz = oracle.halo_accel(st["x"][rows], st["y"][rows], st["z"][rows], halo)
            A = A + np.sqrt(hx * hx + hy * hy + hz * hz)
            e = force_errors(np.stack([st["ax"][rows], st["ay"][rows], st["az"][rows]]),
                             np.stack([ax + hx, ay + hy, az + hz]), A)
            checks.append({"step": step, **e})
            if not (e["eps_cond"] <= 1e-12 and e["eps_rms"] <= 1e-12):
                raise RuntimeError(f"reference run at step {step}: float64 force error {e} above 1e-12")
    else:
        check = None
    ref, _, tref = run("fp64", "o4", 2000, 100, check=check)
    log(f"[bench] reference fp64 o4 dt=5e-4 done in {tref:.1f}s; oracle checks {len(checks)}, worst eps_cond "
        f"{max((c['eps_cond'] for c in checks), default=float('nan')):.2e}")
    runs = {}
    evals_per_step = {"kdk": 1, "o4": 3, "hermite": 1, "rk4": 4}
    for prec in ("fp64", "mixed", "fp32"):
        for scheme, steps in (("kdk", 1000), ("o4", 1000), ("o4", 334), ("hermite", 1000), ("hermite", 500),
                              ("rk4", 250)):
            st, worst, busy = run(prec, scheme, steps, 50)
            dx = np.sqrt(((st["x"] - ref["x"]) ** 2 + (st["y"] - ref["y"]) ** 2 + (st["z"] - ref["z"]) ** 2))
            key = f"{prec}_{scheme}_{steps}"
            runs[key] = {"wall_s": busy, "steps": steps, "evals": steps * evals_per_step[scheme],
                         "pos_err_rms": float(np.sqrt(np.mean(dx ** 2))), "pos_err_max": float(dx.max()), **worst}
            log(f"[bench] {key}: {runs[key]}")
    res = {"metric": "KDK vs fourth-order schemes at equal wall-clock (N=2^17 disk): drift and error",
           "value": runs["mixed_kdk_1000"]["steps"] * float(n) ** 2 / runs["mixed_kdk_1000"]["wall_s"],
           "unit": "pair-interactions/s", "n_gpus": 1, "steps": 1000, "warmup": 0,
           "ms_per_step": 1e3 * runs["mixed_kdk_1000"]["wall_s"] / 1000, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE["mixed"], "data": "synthetic",
           "config": {"workload": "exponential disk N=2^17 + halo, eps=0.02, T=1; reference fp64 O4 dt=5e-4 "
                                  "on the GPU", "n": n,
                      "plans": {k: nb.nbody_plan_get(ctx.h, nb.plan_code(k), n)
                                for k in ("fp64", "mixed", "fp32", "fp64/jerk", "mixed/jerk", "fp32/jerk")}},
           "force_error_rms_vs_fp64": ferr, "runs": runs,
           "reference_check": {"rows": 1024, "gate": 1e-12, "checkpoints": checks},
           "cpu_baseline": None if not checks else {
               "value": cpu["pairs"] / cpu["s"], "unit": "pair-interactions/s", "cores": cpu["threads"],
               "kind": "oracle", "sample": f"1024 rows x {n} sources at each of {len(checks)} checkpoints"}}
    print(json.dumps(res))
    if args.integ_out:
        with open(args.integ_out, "w") as f:
            json.dump(res, f, indent=1)
    ctx.close()


def bench_longrun(args):
    """The paper's precision study (Section 3, Table 2, Figs. 5-7) on the
    completely self-gravitating exponential disk (no halo, eps = 0.02):
    --long-steps leapfrog steps with the paper's ratio of about 4000 steps per
    rotation at the disk's edge, once per precision and once more in float64
    with another summation order (a control: the system is chaotic, so any
    rounding difference grows; what precision adds shows against that).
    Records the largest deviations of P, Lz, E and the centre of mass, their
    time series, and surface-density maps compared with the float64 run."""
    import numpy as np

    import workloads as wl
    from paper_1803_01190_amd import checkpoint
    from paper_1803_01190_amd import longrun as lr
    from paper_1803_01190_amd import nbody as nb

    n, steps, seed, eps = args.long_n, args.long_steps, 3, 0.02
    halo = wl.no_halo()
    period = wl.outer_period(halo=halo)
    dt = period / 4000.0
    ic = wl.make("disk_sg", n, seed)
    ctx = nb.Context(0)
    nb.load_plans(ctx.h)
    if args.long_equilibrium:
        # the disk iterated to the balance of Eqs. (3)-(4) under its own forces
        from paper_1803_01190_amd.equilibrium import equilibrium_disk
        t0 = time.perf_counter()
        ic = equilibrium_disk(ctx.h, ic, eps=eps, seed=seed)
        log(f"[longrun] equilibrium initial conditions in {time.perf_counter() - t0:.1f}s")
    grid = lr.Grid(256, 256, -6.0, -6.0, 12.0 / 256)
    maps_at = [steps * k // 10 for k in range(11)]
    alt_plan = {"R": 1, "block": 256, "split": 3, "jsrc": 0}  # a split no tuned plan uses
    os.makedirs(args.out_dir, exist_ok=True)
    recs, out = {}, {}
    for name in args.long_runs.split(","):
        prec = "fp64" if name == "fp64_alt" else name
        prm = nb.Params(eps=eps, prec=nb.PREC[prec])
        plan = alt_plan if name == "fp64_alt" else None
        t0 = time.perf_counter()
        last = [t0]

        def progress(done, rec, name=name, t0=t0, last=last):
            # every 1000 steps, and at least once a minute for large systems
            now = time.perf_counter()
            if done % 1000 == 0 or done == steps or now - last[0] >= 60.0:
                last[0] = now
                dv = rec.deviations()
                log(f"[longrun] {name} step {done}/{steps} ({now - t0:.0f}s) "
                    f"dE {dv['dE_rel'][-1]:.2e} dL {dv['dL_rel'][-1]:.2e} dP {dv['dP_abs'][-1]:.2e}")

        # a run may be cut into pieces (--stop-at, then --resume-dir with the
        # saved piece); pieces are compact snapshots (positions, velocities
        # and the common mass), whose accelerations are recomputed on load
        # under the run's plan, which gives the bits the run carried
        run_ic, resume = ic, None
        if args.resume_dir:
            rstem = os.path.join(args.resume_dir, f"resume_{name}_{n}")
            if plan is not None:
                nb.nbody_plan_set(ctx.h, prm.prec, n, plan)
            st, _, _, step, _ = checkpoint.load(rstem + "_state.npz", ctx=ctx.h)
            run_ic = st.numpy()
            del st
            resume = (lr.Record.load(rstem), step)
            log(f"[longrun] {name}: resuming at step {step}")
        deadline = None if args.stop_after_s is None else T_START + args.stop_after_s
        rec = lr.run(ctx.h, run_ic, prm, dt, steps, every=50, maps_at=maps_at, grid=grid, plan=plan,
                     progress=progress, resume=resume, stop_at=args.stop_at, deadline=deadline)
        if rec.done < steps:
            stem = os.path.join(args.out_dir, f"resume_{name}_{n}")
            checkpoint.save(stem + "_state.npz", nb.System.from_arrays(rec.final), prm, step=rec.done,
                            compact=True)
            rec.save(stem)
            log(f"[longrun] {name}: stopped at step {rec.done}, saved {stem}*")
        recs[name] = rec
        out[name] = {**rec.table2(), "wall_s": rec.busy_s, "evals": rec.evals, "done": rec.done,
                     "pair_interactions_per_s": lr.interactions_per_s(n, rec)}
        log(f"[longrun] {name}: {out[name]}")
    ref = recs.get("fp64")
    maps = {}
    if ref is not None and all(rec.done == steps for rec in recs.values()):
        for name, rec in recs.items():
            if name == "fp64":
                continue
            maps[name] = {str(k): lr.compare_maps(ref.maps[k], rec.maps[k]) for k in maps_at}
        maps["fp64_m2"] = {str(k): lr.nonaxisymmetry(ref.maps[k], grid) for k in maps_at}
    series = {name: {"step": rec.steps, **{k: v.tolist() for k, v in rec.deviations().items()}}
              for name, rec in recs.items()}
    with open(os.path.join(args.out_dir, f"longrun_{n}.json"), "w") as f:
        json.dump({"n": n, "dt": dt, "steps": steps, "eps": eps, "period": period, "table2": out,
                   "maps": maps, "series": series}, f)
    np.savez_compressed(os.path.join(args.out_dir, f"maps_{n}.npz"),
                        **{f"{name}_{k}": rec.maps[k] for name, rec in recs.items() for k in maps_at
                           if k in rec.maps})
    head = "mixed" if "mixed" in out else next(iter(out))
    res = {"metric": "10^4-step conservation (Table 2 quantities) and density-map deviation vs float64",
           "value": out[head]["pair_interactions_per_s"], "unit": "pair-interactions/s", "n_gpus": 1,
           "steps": steps, "warmup": 0, "ms_per_step": 1e3 * out[head]["wall_s"] / steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[
               "fp64" if head == "fp64_alt" else head], "data": "synthetic",
           "config": {"workload": f"self-gravitating exponential disk N={n} (no halo), eps={eps}, "
                                  f"KDK dt={dt:.6g} (outer period / 4000), seed {seed}"
                                  + (", iterated to equilibrium" if args.long_equilibrium else ""), "n": n},
           "table2": out, "maps": maps}
    print(json.dumps(res))
    ctx.close()


def bench_hermite(args):
    """The fourth-order Hermite step at N = 2^20 on the headline disk (eps =
    0.02, halo): one acceleration-and-jerk pair pass per step with the
    corrector fused, timed per precision like the KDK step; errors of a and j
    against the oracle on sampled rows."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    dev = torch.device("cuda:0")
    n, dt, eps = args.n, 1e-3, 0.02
    halo = wl.default_halo()
    ic = wl.exp_disk(n, 2)
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    ctx = nb.Context(0)
    nb.load_plans(ctx.h)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n, size=min(args.sample_rows, n), replace=False))
    rows_t = torch.as_tensor(rows, device=dev)
    results = {}
    for prec in precs:
        prm = nb.Params(G=1.0, eps=eps, prec=nb.PREC[prec], halo=True, halo_v2=halo.v2, halo_rc=halo.rc)
        s = nb.System.from_arrays(ic, device=dev)
        nb.nbody_accel_jerk(ctx.h, s, prm)
        aj0 = torch.stack([s[k][rows_t] for k in ("ax", "ay", "az", "jx", "jy", "jz")]).cpu().numpy()
        for _ in range(args.warmup):
            nb.nbody_step_hermite(ctx.h, s, prm, dt, 1)
        d0 = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
        torch.cuda.synchronize()
        nb.nbody_profile_read(ctx.h)
        nb.nbody_profile_enable(ctx.h, True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            nb.nbody_step_hermite(ctx.h, s, prm, dt, 1)
            evs[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        nb.nbody_profile_enable(ctx.h, False)
        prof = nb.nbody_profile_read(ctx.h)
        d1 = nb.diag_dict(nb.nbody_diag(ctx.h, s, prm))
        step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        if prec == precs[0] and args.steps < MIN_LATENCY_SAMPLES and not args.profile_run:
            # more per-step latency samples for p50/p99, after the timed region
            extra = MIN_LATENCY_SAMPLES - args.steps
            ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(extra + 1)]
            ev2[0].record()
            for k in range(extra):
                nb.nbody_step_kdk(ctx.h, s, prm, dt, 1)
                ev2[k + 1].record()
            torch.cuda.synchronize()
            step_ms += [ev2[k].elapsed_time(ev2[k + 1]) for k in range(extra)]
        inter = float(n) * float(n)
        pair_ms = prof["accel_ms"] / max(prof["accel_launches"], 1)
        tflops = JERK_FLOPS_PER_INTERACTION * inter / (pair_ms * 1e-3) / 1e12
        results[prec] = {
            "value": args.steps * inter / wall, "ms_per_step": 1e3 * wall / args.steps,
            "latency_ms": {"p50": percentile(step_ms, 0.5), "p99": percentile(step_ms, 0.99)},
            "pair_kernel_ms": pair_ms, "pair_launches": prof["accel_launches"],
            "plan": nb.nbody_plan_get(ctx.h, nb.PREC[prec] | nb.NB_PLAN_JERK, n),
            "update_ms_per_step": prof["update_ms"] / max(args.steps, 1), "achieved_tflops": tflops,
            "drift": {"dE_rel": abs(d1["E"] - d0["E"]) / abs(d0["E"]),
                      "dLz_rel": abs(d1["Lz"] - d0["Lz"]) / abs(d0["Lz"]), "steps": args.steps},
            "_aj0": aj0,
        }
        log(f"[hermite] {prec}: {results[prec]['value']:.4e} pair-int/s, {1e3 * wall / args.steps:.1f} ms/step, "
            f"pair kernel {pair_ms:.1f} ms ({tflops:.1f} TFLOP/s at {JERK_FLOPS_PER_INTERACTION} flop/pair)")
        del s
        torch.cuda.empty_cache()
    cpu, errs = None, {}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        cores = oracle.max_threads()
        t0 = time.perf_counter()
        ref = oracle.accel_jerk(ic, 1.0, eps, oracle.Halo(halo.v2, halo.rc), want_scale=True, rows=rows)
        el = time.perf_counter() - t0
        cpu = {"value": rows.size * float(n) / el, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
               "sample": f"{rows.size} seeded rows of the N=2^20 disk, acceleration and jerk over all {n} "
                         f"sources (float64, {el:.1f} s on {cores} threads)"}
        A, J = ref[6], ref[7]
        for prec, r in results.items():
            g = r["_aj0"]
            da = np.sqrt(((g[:3] - np.stack(ref[:3])) ** 2).sum(0))
            dj = np.sqrt(((g[3:] - np.stack(ref[3:6])) ** 2).sum(0))
            errs[prec] = {"a_cond": float(np.max(da / A)), "j_cond": float(np.max(dj / J))}
        log(f"[hermite] cpu oracle {cpu['value']:.3e} pair-int/s; errors {errs}")
    head = precs[0]
    r0 = results[head]
    out = {
        "metric": "pair-interactions/s at N=2^20, fourth-order Hermite step (acceleration and jerk per pair)",
        "value": r0["value"], "unit": "pair-interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r0["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[head], "data": "synthetic",
        "config": {"workload": f"exponential stellar disk N={n} + fixed isothermal halo, eps={eps}, "
                               f"Hermite dt={dt}", "n": n, "integrator": "hermite", "precision": head},
        "latency_ms": r0["latency_ms"],
        "roofline": {"bound": "alu", "achieved": r0["achieved_tflops"], "peak": PEAK_TFLOPS[head],
                     "unit": "TFLOP/s", "frac": r0["achieved_tflops"] / PEAK_TFLOPS[head], "traffic": None,
                     "kernel": ("acceleration and jerk in spatial order (k_pair_jerk_local, with its "
                                "ordering kernels)" if r0["plan"].get("jsrc") == 2 else
                                "acceleration and jerk (k_pair_jerk)"),
                     "flops_per_interaction": JERK_FLOPS_PER_INTERACTION, "interactions_per_launch": inter},
        "cpu_baseline": cpu, "errors": errs or None,
        "per_precision": {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")} for k, v in results.items()},
    }
    print(json.dumps(out))
    ctx.close()


# The paper's Table 1: one KDK step on one Tesla K80 GPU, seconds, for
# N = 128K ... 8192K particles (N x 1024), single and double precision.
PAPER_TABLE1_K80 = {
    "n_k": [128, 256, 512, 1024, 2048, 4096, 8192],
    "sp_s": [0.4, 1.7, 6.9, 27.4, 109.6, 438.0, 1754.0],
    "dp_s": [0.9, 3.7, 15.0, 60.0, 240.0, 960.0, 3840.0],
}


def bench_scaling(args):
    """One KDK step of the disk (eps = 0.02, halo) for N = 2^17 ... 2^max on
    one GPU, per precision: the single-GPU columns of the paper's Table 1
    (whose disk model differs; its K80 times are listed as context).  Sizes
    without a tuned plan are autotuned first (bounded budget)."""
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    ctx = nb.Context(0)
    nb.load_plans(ctx.h)
    halo = wl.default_halo()
    table = nb.read_plans()
    rows = []
    for log2n in range(17, args.scaling_max_log2 + 1):
        n = 1 << log2n
        ic = wl.exp_disk(n, 2)
        for prec in precs:
            p = nb.PREC[prec]
            if str(log2n) not in table.get(prec, {}):
                nb.nbody_autotune(ctx.h, p, n, 1500.0)
            plan = nb.nbody_plan_get(ctx.h, p, n)
            prm = nb.Params(eps=0.02, prec=p, halo=True, halo_v2=halo.v2, halo_rc=halo.rc)
            s = nb.System.from_arrays(ic)
            nb.nbody_accel(ctx.h, s, prm)  # a(t0); also warms up the same kernel and plan
            steps = max(1, min(args.steps, int(2e12 // (float(n) * n)) + 1))
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            nb.nbody_step_kdk(ctx.h, s, prm, 1e-3, steps)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / steps
            rows.append({"n": n, "prec": prec, "step_s": t, "pair_interactions_per_s": float(n) * n / t,
                         "plan": plan, "steps": steps})
            log(f"[scaling] N=2^{log2n} {prec}: {t:.4f} s/step, {float(n) * n / t:.3e} pair-int/s, plan {plan}")
            del s
            torch.cuda.empty_cache()
    head = "mixed" if "mixed" in precs else precs[0]
    top = [r for r in rows if r["prec"] == head][-1]
    res = {"metric": "one KDK step time vs N on one GPU (the paper's Table 1, single-GPU columns)",
           "value": top["pair_interactions_per_s"], "unit": "pair-interactions/s", "n_gpus": 1,
           "steps": top["steps"], "warmup": 0, "ms_per_step": 1e3 * top["step_s"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[head], "data": "synthetic",
           "config": {"workload": f"exponential stellar disk N=2^17..2^{args.scaling_max_log2} + fixed isothermal "
                                  "halo, eps=0.02, KDK dt=1e-3", "precisions": precs},
           "rows": rows, "paper_table1_k80_one_gpu": PAPER_TABLE1_K80}
    print(json.dumps(res))
    ctx.close()


def bench_serving(args):
    """Poisson request stream through the continuous-batching loop: N
    log-uniform in [2^lo, 2^hi] (default [2^12, 2^20]), steps uniform in
    [10, 1000], Plummer or disk with equal odds, mixed with 10% FP64
    (--serve-* options narrow it).  The capacity mu (requests/s with every
    request arriving at once) is measured first unless --capacity gives it;
    then each rate of --rates (fractions of mu) runs the same requests with
    Poisson arrival times scaled to that rate.  Reports completed requests/s,
    pair-interactions/s and p50/p99 latency (arrival to result on the host)."""
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb
    from paper_1803_01190_amd.serving import GpuBackend, Request, Scheduler

    ctx = nb.Context(0)
    nb.load_plans(ctx.h)
    nreq = args.requests
    lo, _, hi = args.serve_log2.partition("-")
    slo, _, shi = args.serve_steps.partition("-")
    lo, hi, slo, shi = int(lo), int(hi), int(slo), int(shi)

    # the requests' initial conditions are prepared by the client before
    # they arrive (outside the timed runs); arrival times are rescaled per rate
    base = wl.request_stream(nreq, seed=5, rate=1.0, lo_log2=lo, hi_log2=hi, steps_lo=slo, steps_hi=shi,
                             fp64_fraction=0.1)
    ics = [wl.make(r["model"], r["n"], r["seed"]) for r in base]
    work = sum(float(r["n"]) ** 2 * r["steps"] for r in base)
    log(f"[bench] serving: {nreq} requests, N in [2^{lo}, 2^{hi}], steps in [{slo}, {shi}], "
        f"{work:.3e} pair-interactions in all")

    def make(rate):
        return [Request(id=r["id"], t_arrive=r["t_arrive"] / rate, n=r["n"], steps=r["steps"], model=r["model"],
                        fp64=r["fp64"], seed=r["seed"], ic=ics[k]) for k, r in enumerate(base)]

    budget = 64 << 30
    graph = not args.no_graph
    last = [0.0]

    def progress(info, tag=""):
        if info["t"] - last[0] >= 30.0:
            last[0] = info["t"]
            log(f"[serving{tag}] t={info['t']:.0f}s done {info['done']}/{nreq} active {info['active']} "
                f"waiting {info['waiting']} pending {info['pending']} HBM {info['used_bytes'] / 2**30:.1f} GiB")

    def run(rate, tag):
        last[0] = 0.0
        be = GpuBackend(ctx.h, keep_state=False, graph=graph, diagnostics=False)
        sch = Scheduler(be, hbm_budget=budget, max_tick_steps=25, progress=lambda i: progress(i, tag))
        smry = sch.run(make(rate)).summary()
        be.close()
        return smry, be.plan

    plan = None
    if args.capacity:
        mu, cap = args.capacity, None
    else:
        cap, plan = run(1e9, " capacity")
        mu = cap["requests_per_s"]
        log(f"[bench] serving capacity {mu:.4f} req/s ({cap})")
    sweep = []
    for frac in [float(f) for f in args.rates.split(",") if f]:
        smry, plan = run(frac * mu, f" {frac:.2f} mu")
        smry["rate_req_per_s"] = frac * mu
        smry["rate_frac"] = frac
        sweep.append(smry)
        log(f"[bench] serving rate {frac:.2f} mu: {smry}")
    torch.cuda.synchronize()
    head = sweep[len(sweep) // 2] if sweep else cap
    res = {"metric": "serving throughput (requests/s, pair-interactions/s) and p50/p99 latency",
           "value": head["interactions_per_s"], "unit": "pair-interactions/s", "n_gpus": 1,
           "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPE["mixed"], "data": "synthetic",
           "config": {"workload": f"{nreq} Poisson-arriving requests per rate, N log-uniform in [2^{lo}, 2^{hi}], "
                                  f"steps uniform in [{slo}, {shi}], Plummer or disk, 10% FP64, HBM budget 64 GiB",
                      "capacity_req_per_s": mu, "graph_replay": graph,
                      "batch_plan": plan,
                      "requests": [{k: r[k] for k in ("n", "steps", "model", "fp64")} for r in base]},
           "latency_s": head["latency_s"], "capacity": cap, "sweep": sweep}
    print(json.dumps(res))
    if args.serve_out:
        with open(args.serve_out, "w") as f:
            json.dump(res, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
