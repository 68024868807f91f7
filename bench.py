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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s at N=2^20 (FP64 vs mixed @ stated err); p50/p99 latency"
FLOPS_PER_INTERACTION = 20  # conventional count for the softened pair term
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3, "fp32": 157.3}  # MI355X vector peaks
DTYPE = {"fp64": "f64", "mixed": "f32 pair / f64 accumulate+state", "fp32": "f32"}
KERNEL_SOURCES = ["paper_1803_01190_amd/csrc/accel.hip", "paper_1803_01190_amd/csrc/nbody_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(prec: str):
    """HBM bytes per pair-sum launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
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
    ap.add_argument("--sample-rows", type=int, default=8192,
                    help="oracle rows (each summed over all N) for the CPU baseline and force errors")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plans-in", default=None,
                    help="plan-cache JSON ({arch: {prec: {log2n: plan}}}); default: the committed "
                         "tuned_plans.json when it has this size, else autotune")
    ap.add_argument("--retune", action="store_true", help="autotune even if a cached plan exists")
    ap.add_argument("--plans-out", default=None, help="write the plans used in plan-cache form")
    ap.add_argument("--profile-run", action="store_true",
                    help="run for counter collection: no CPU baseline, plus a copy kernel of "
                         "known size to calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU target split is a design in DESIGN.md, not a run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1803_01190_amd import nbody as nb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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
        wall = w1 - w0
        inter = float(n) * float(n)
        rate = args.steps * inter / wall
        accel_ms = prof["accel_ms"] / max(prof["accel_launches"], 1)
        tflops = FLOPS_PER_INTERACTION * inter / (accel_ms * 1e-3) / 1e12
        m_tot = float(np.sum(ic["m"]))
        results[prec] = {
            "value": rate,
            "ms_per_step": 1e3 * wall / args.steps,
            "latency_ms": {"p50": percentile(step_ms, 0.5), "p99": percentile(step_ms, 0.99)},
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
    traffic = load_traffic(head)
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
            "kernel": "pair sum (k_pair)",
            "flops_per_interaction": FLOPS_PER_INTERACTION,
            "interactions_per_launch": float(n) * float(n),
        },
        "cpu_baseline": cpu,
        "force_error": force_err or None,
        "per_precision": {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")}
                          for k, v in results.items()},
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
