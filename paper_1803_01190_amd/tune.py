"""Regenerate the plan cache ``tuned_plans.json`` from the library's own
autotuner: every kernel class and precision is tuned on the exponential disk
of the headline workload (eps = 0.02, halo) at each size class, over every
candidate plan on the whole system (``nbody_autotune_sys``), and the batch
plan on the batched workload (256 systems, N log-uniform in [2^10, 2^16];
``nbody_batch_autotune``).  The file maps
``{arch: {"prec[/class]": {ceil(log2 n): plan}}}``.

    python -m paper_1803_01190_amd.tune --log2n 17-20 --out tuned_plans.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import nbody as nb


def _range(text: str) -> list[int]:
    lo, _, hi = text.partition("-")
    return list(range(int(lo), int(hi or lo) + 1))


def main(argv=None) -> int:
    import numpy as np
    import torch

    import workloads as wl

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--log2n", default="17-20", help="size classes, e.g. 17-20")
    ap.add_argument("--precs", default="mixed,fp64,fp32")
    ap.add_argument("--classes", default="accel,jerk,potential", help="kernel classes (potential: fp64 only)")
    ap.add_argument("--batch", action="store_true", help="also tune the batch plan on the batched workload")
    ap.add_argument("--budget-ms", type=float, default=0.0, help="per key (0: every candidate)")
    ap.add_argument("--out", default=nb.TUNED_PLANS)
    ap.add_argument("--merge", action="store_true", help="keep the file's entries that are not re-tuned")
    ap.add_argument("--start", default=None,
                    help="plan cache whose plans are pinned first (each key's first candidate)")
    ap.add_argument("--arch", default="gfx950")
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "tuning needs the GPU"

    table = nb.read_plans(args.out, args.arch) if args.merge else {}
    h = wl.default_halo()
    ctx = nb.Context(0)
    if args.start:
        # each key's plan in this cache is its first candidate
        nb.load_plans(ctx.h, args.start, args.arch)
    try:
        for log2n in _range(args.log2n):
            n = 1 << log2n
            ic = wl.exp_disk(n, 2)
            for cls in args.classes.split(","):
                for prec in args.precs.split(","):
                    if cls == "potential" and prec != "fp64":
                        continue  # the diagnostics' potential pass is float64
                    key = prec if cls == "accel" else f"{prec}/{cls}"
                    prm = nb.Params(eps=0.02, prec=nb.PREC[prec], halo=True, halo_v2=h.v2, halo_rc=h.rc)
                    s = nb.System.from_arrays(ic)
                    t0 = time.perf_counter()
                    plan = nb.nbody_autotune_sys(ctx.h, nb.plan_code(key), s, prm, args.budget_ms)
                    print(f"[tune] {key} 2^{log2n}: {plan} ({time.perf_counter() - t0:.1f}s)", file=sys.stderr,
                          flush=True)
                    table.setdefault(key, {})[str(log2n)] = plan
                    del s
        if args.batch:
            mix = wl.batch_mix(256, 4)
            off = mix["off"]
            B = len(off) - 1
            prms = [nb.Params(eps=0.01 if mix["kind"][k] == "plummer" else 0.02, prec=nb.NB_MIXED,
                              halo=mix["kind"][k] == "disk", halo_v2=h.v2, halo_rc=h.rc) for k in range(B)]
            b = nb.nbody_batch_create(ctx.h, off, prms, [1e-3] * B)
            try:
                s = nb.System.from_arrays(mix)
                t0 = time.perf_counter()
                plan = nb.nbody_batch_autotune(ctx.h, b, s, args.budget_ms)
                nmax = int(np.diff(off).max())
                log2 = max(0, (nmax - 1).bit_length())
                print(f"[tune] mixed/batch (largest system 2^{log2}): {plan} ({time.perf_counter() - t0:.1f}s)",
                      file=sys.stderr, flush=True)
                table.setdefault("mixed/batch", {})[str(log2)] = plan
            finally:
                nb.nbody_batch_destroy(ctx.h, b)
    finally:
        ctx.close()
    ordered = {k: dict(sorted(v.items(), key=lambda kv: int(kv[0]))) for k, v in sorted(table.items())}
    with open(args.out, "w") as f:
        json.dump({args.arch: ordered}, f, indent=1)
        f.write("\n")
    print(f"[tune] wrote {args.out}", file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
