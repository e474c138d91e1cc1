#!/usr/bin/env python
"""Throughput of the RK2 substep on one MI355X.

Workload (default): the Rayleigh-Taylor configuration 512 x 385 x 512
(Fourier x B-spline x Fourier modes, 768 x 768 dealiased x-z grid), FP64,
At = 0.925 (density ratio 25.67), Re = 1024, k_f = 4 fixed-point iterations,
seeded synthetic fields (no dataset).  A step is one substep of the method
(all phases: m^d, R_z, k_f iterations, m^c, fluxes, RHS, RK2 update); stages
alternate n, ', n, ...  Inputs are resident in HBM before the timed region.

Prints one JSON line with substeps/s, the roofline of the dominant kernel
class (HIP events on the library's stream over the timed region) and the CPU
oracle baseline.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CLASS_NAMES = ("eval_zinv", "xpass", "zfwd", "proj", "solveA", "rhs")


def substep_model_bytes(w, kf):
    """Algorithmic HBM bytes of one substep under the dataflow model of the
    method: (87 + 16 k_f) spectral-field passes of N1/2 (N3-1) n2 complex128."""
    s = (w.n1 // 2) * (w.n3 - 1) * w.n2 * 16.0
    return (87 + 16 * kf) * s


def cpu_baseline(full):
    """The oracle, untouched, on a bounded sample: one substep of the same
    workload recipe at 128 x 97 x 128 (192 x 192 grid), scaled to the full
    size by the ratio of transform work N1 N3 n2 log2(M1 M3)."""
    from threadpoolctl import threadpool_info

    from oracle.lmvd import Config, Plan as OPlan, substep
    from paper_2206_09878_amd.workloads import make_inputs, workload
    w = workload(full.name, n=128, n2=97)
    inp = make_inputs(w, seed=2)
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    cfg = Config(w.n1, w.n3, w.n2, w.order, w.m1, w.m3, w.L1, w.L2, w.L3, w.breakpoints, w.dt, w.mu,
                 w.rhoD, w.g, w.rho_l, w.rho_h, w.beta_n, w.beta_p, w.kf)
    op = OPlan(cfg)
    t0 = time.perf_counter()
    substep(op, st, 0, hist=inp["hist"])
    t = time.perf_counter() - t0

    def work(x):
        return x.n1 * x.n3 * x.n2 * math.log2(x.m1 * x.m3)

    ratio = work(full) / work(w)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": 1.0 / (t * ratio), "unit": "substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"one oracle substep of the {full.name} recipe at 128x97x128 (192x192 grid): "
                      f"{t:.1f} s, scaled by the transform-work ratio {ratio:.1f} to "
                      f"{full.n1}x{full.n2}x{full.n3}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rt512")
    ap.add_argument("--plane-batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-class", choices=CLASS_NAMES, default=None,
                    help="time this kernel class instead of detecting the dominant one")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs the substep on one GPU only; multi-GPU sharding is a design "
              "(see the design notes), not a run. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2206_09878_amd.lmvd import Plan, Stepper
    from paper_2206_09878_amd.workloads import make_inputs, workload

    torch.cuda.set_device(0)
    w = workload(args.workload)
    plan = Plan(w, plane_batch=args.plane_batch)
    stepper = Stepper(plan, make_inputs(w, seed=2, stage=0), stage=0)
    for _ in range(args.warmup):
        stepper.substep()
    torch.cuda.synchronize()

    # dominant kernel class: one untimed substep per class with its launches timed
    totals = {}
    if args.kernel_class is None:
        for cls in range(len(CLASS_NAMES)):
            plan.profile_start(cls)
            stepper.substep()
            ms, n, b = plan.profile_stop()
            totals[cls] = ms
        dom = max(totals, key=totals.get)
    else:
        dom = CLASS_NAMES.index(args.kernel_class)
    torch.cuda.synchronize()

    # timed region
    plan.profile_start(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stepper.substep()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, klaunch, kbytes = plan.profile_stop()

    value = args.steps / elapsed
    achieved = kbytes / (kms * 1e-3) / 1e9
    model = substep_model_bytes(w, w.kf)
    out = {
        "metric": "RK substeps/s at 512x385x512 FP64",
        "value": value,
        "unit": "substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: Rayleigh-Taylor At=0.925, {w.n1}x{w.n2}x{w.n3} modes, "
                               f"{w.m1}x{w.m3} dealiased x-z grid, k_f={w.kf}, stages n/' alternating",
                   "kf": w.kf, "plane_batch": args.plane_batch or w.n2},
        "roofline": {"bound": "hbm", "kernel": CLASS_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "launches": klaunch, "avg_launch_ms": kms / max(klaunch, 1),
                     "share_of_substep": (totals[dom] / sum(totals.values())) if totals else None},
        "substep_roofline": {"model_bytes_per_substep": model,
                             "frac": model * value / (HBM_PEAK_GBS * 1e9)},
        "kernel_class_ms_per_substep": {CLASS_NAMES[c]: totals[c] for c in totals},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
