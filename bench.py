#!/usr/bin/env python
"""Throughput of the RK2 substep on one MI355X.

Workload (default): the Rayleigh-Taylor configuration 512 x 385 x 512
(Fourier x B-spline x Fourier modes, 768 x 768 dealiased x-z grid), FP64,
At = 0.925 (density ratio 25.67), Re = 1024, k_f = 4 fixed-point iterations,
seeded synthetic fields (no dataset).  A step is one substep of the method
(all phases: m^d, R_z, k_f iterations, m^c, fluxes, RHS, RK2 update); stages
alternate n, ', n, ...  Inputs are resident in HBM before the timed region.

Prints one JSON line with substeps/s (timed with no hook active), the
roofline of the dominant kernel (its launches bracketed by HIP events on the
library's stream in a pass of its own, algorithmic bytes from the method's
spectral-field dataflow) and the CPU oracle baseline.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
    python bench.py --workload batch64     (64 small uneven instances, one HIP graph)
    python bench.py --workload adjoint96   (gradient of the 96^3 workload: adjoint/forward time)
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2206_09878_amd", "csrc", "lmvd.hip")
TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def class_names():
    from paper_2206_09878_amd.lmvd import Plan
    return Plan.KERNEL_CLASSES


def kernel_symbol(cls: str, w) -> str:
    """Kernel symbol a class launches on the register-FFT sizes (as rocprofv3 names it)."""
    m1, m3 = w.m1, w.m3
    return {
        "zinv": f"k_zinv_w<{m3}, true>" if m3 == 768 else f"k_zinv_r<{m3}, true>",
        "zfwd": f"k_zfwd_w<{m3}>" if m3 == 768 else f"k_zfwd_r<{m3}>",
        "xpass_rz": f"k_xpair<0, {m1}>", "xpass_rhot": f"k_xline<1, {m1}>", "xpass_l": f"k_xline<2, {m1}>",
        "xpass_vel": f"k_xpair_w2<3, {m1}>", "mc": "k_mc<7, 7, 6, true>", "md": "k_prologue<7, 7, 8>", "proj": "k_proj<0>, k_proj3",
        "proj_zt": "k_proj<1>, k_proj<2>", "values": "k_values",
        "flux": "k_flux<0, 8, 6>, k_flux<1, 8, 6>", "rhs": "k_rhs_fluct, k_rhs_mean",
        "zfilt": (f"k_zfilt_w<{m3}>" if m3 == 768 else f"k_zfilt_r<{m3}>") + ", k_wall",
    }.get(cls, cls)


def source_digest() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


KIND = {"rt512": "Rayleigh-Taylor At=0.925, multimode interface", "mixing128": "temporal mixing layer",
        "adjoint96": "temporal mixing layer", "small": "broadband random fields"}


def counter_traffic(cls: str, w):
    """HBM bytes per launch of `cls` from the committed rocprofv3 counter summary, or None when
    there is none for this class and workload or the kernel source changed since it was taken."""
    path = os.path.join(TRAFFIC_DIR, f"traffic_{cls}_{w.name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_digest():
        return None
    return t["fetch_kib_per_dispatch"] * 1024.0 * t["fetch_scale"] + \
        t["write_kib_per_dispatch"] * 1024.0 * t["write_scale"]


def sfield_bytes(w):
    """One spectral field: N1/2 (N3-1) n2 complex128."""
    return (w.n1 // 2) * (w.n3 - 1) * w.n2 * 16.0


def substep_model_bytes(w, kf):
    """HBM bytes of one substep under the reference dataflow of the method:
    (87 + 16 k_f) spectral-field passes."""
    return (87 + 16 * kf) * sfield_bytes(w)


def model_bytes_per_substep(cls, w, kf):
    """Algorithmic bytes of one kernel class per substep in the same dataflow, for the classes whose
    spectral-field I/O the dataflow fixes: the m^c solve of an iterate reads the rho_t values and writes
    the three m^c value fields (4 passes); the final one also reads the three m^d value fields and writes
    m = m^d + m^c (7 passes); k_f + 1 launches per substep."""
    if cls == "mc":
        return (4 * kf + 7) * sfield_bytes(w)
    return None


def hbm_ceiling(gib, reps=10):
    """Achieved bandwidth of plain streaming kernels (torch's copy, fill, sum and add) over
    GIB-sized FP64 buffers, timed with HIP events: the practical ceiling for the substep's kernels."""
    import torch
    n = int(gib * 2**30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    nb = 8.0 * n
    return {"buffer_gib": gib, "unit": "TB/s",
            "copy_read1_write1": 2 * nb / timed(lambda: c.copy_(a)) / 1e12,
            "fill_write1": nb / timed(lambda: c.fill_(1.5)) / 1e12,
            "sum_read1": nb / timed(lambda: a.sum()) / 1e12,
            "add_read2_write1": 3 * nb / timed(lambda: torch.add(a, b, out=c)) / 1e12}


def bench_batch(args, count=64, nsub=4):
    """64 independent small instances of uneven sizes: all of them advanced by one
    HIP graph launch (nsub substeps each), against the same substeps launched one
    by one on the plain path, instance after instance, on one stream."""
    import torch

    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    from paper_2206_09878_amd.workloads import batch_workloads, make_inputs
    ws = batch_workloads(count)
    st = [Stepper(Plan(w), make_inputs(w, seed=w.extra["seed"], stage=0), stage=0) for w in ws]

    def eager():
        for s in st:
            for _ in range(nsub):
                s.substep()

    def timed(fn, k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    # the graph with the default z tile, then with the tiles the graph autotuner picks (its tries
    # advance the instances like warm-up launches)
    t0 = time.perf_counter()
    g = GraphBatch(st, nsub=nsub)
    build_s = time.perf_counter() - t0
    for _ in range(max(args.warmup, 1)):
        g.launch()
    t_default = timed(g.launch, args.steps)
    t0 = time.perf_counter()
    tiles, _ = g.autotune(launches=3)
    tune_s = time.perf_counter() - t0
    chosen = {}
    for w, t in zip(ws, tiles):
        chosen[str(w.m3)] = t
    # the candidates' times for one instance of each z size alone (lmvd_autotune on a copy of its plan)
    alone = {}
    for m3 in sorted({w.m3 for w in ws}):
        w = next(x for x in ws if x.m3 == m3)
        _, times = Plan(w).autotune()
        alone[str(m3)] = {str(code): round(ms, 4) for code, ms in zip(Plan.TILE_CODES, times) if ms > 0}
    for _ in range(max(args.warmup, 1)):
        g.launch()
        eager()
    tg = timed(g.launch, args.steps)
    te = timed(eager, args.steps)
    subs = count * nsub * args.steps
    pts = sum(w.m1 * w.m3 * w.n2 for w in ws) * nsub * args.steps
    return {"metric": f"instance-substeps/s, {count} uneven instances in one HIP graph", "value": subs / tg,
            "unit": "instance-substeps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * tg / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"batch{count}: N1, N3 in {{32,48,64,96}}, n2 in {{33,49,65,97}}, density ratio "
                                   f"U[2,25], seeds 1000..{999 + count}; a step = one graph launch = {nsub} substeps "
                                   f"of every instance", "kf": ws[0].kf},
            "grid_point_substeps_per_s": pts / tg,
            "one_by_one": {"value": subs / te, "ms_per_step": 1e3 * te / args.steps,
                           "grid_point_substeps_per_s": pts / te},
            "graph_speedup": te / tg, "graph_build_s": build_s,
            "autotune": {"z_tile_code_per_size": chosen, "tile_code": "D + 8 V (V: line plan, D: divisor)",
                         "tune_s": tune_s, "default_tile_value": subs / t_default,
                         "speedup_over_default_tile": t_default / tg, "alone_ms_per_code": alone}}


def bench_adjoint(args, steps=20, every=5):
    """The adjoint workload: 96 x 97 x 96 (density 1 -> 7 layer), 20 RK steps, objective the domain-
    averaged kinetic energy at the final time, gradient with respect to the initial z through the
    library's adjoint substep with checkpointed recomputation every 5 steps.  A step = one forward +
    backward of the whole workload; the native forward (the same 41 substeps on the plain path) is
    timed beside it."""
    import torch

    from paper_2206_09878_amd.adjoint import final_kinetic_energy, rollout
    from paper_2206_09878_amd.lmvd import Plan, Stepper
    from paper_2206_09878_amd.workloads import make_inputs, workload
    w = workload("adjoint96")
    p = Plan(w)
    inp = make_inputs(w, seed=98, stage=0)
    st0 = {k: p.to_dev(inp[k]) for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    hist0 = [p.to_dev(h) for h in inp["hist"]]

    def native():
        s = Stepper(p, inp, stage=0)
        for _ in range(2 * steps + 1):
            s.substep()

    def adjoint():
        z0 = st0["z"].clone().requires_grad_(True)
        state, hist = rollout(p, dict(st0, z=z0), hist0, steps=steps, checkpoint_every=every)
        final_kinetic_energy(p, state, hist).backward()
        return z0.grad

    def timed(fn, k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / k

    for _ in range(max(args.warmup, 1)):
        native()
        adjoint()
    k = max(1, min(args.steps, 5))
    t_nat = timed(native, k)
    t_adj = timed(adjoint, k)
    return {"metric": "adjoint/forward time, 96x97x96 FP64, 20 RK steps checkpointed every 5", "value": t_adj / t_nat,
            "unit": "ratio", "n_gpus": 1, "steps": k, "warmup": args.warmup, "ms_per_step": 1e3 * t_adj,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "adjoint96: temporal mixing layer, density ratio 7, 96x97x96 modes, 144x144 grid, "
                                   "k_f=4, 20 RK steps (40 substeps) + the objective's substep; gradient of the "
                                   "final kinetic energy in the initial z; a step = forward + backward", "kf": w.kf},
            "native_forward_ms": 1e3 * t_nat, "forward_plus_backward_ms": 1e3 * t_adj}


def cpu_baseline(full, n2=9):
    """The oracle, untouched, on a bounded sample: one stage-n substep of the same workload at full
    horizontal size with n2 = 9 B-spline coefficients, scaled linearly in n2 to the full size (every
    step of the substep is per y-plane or per y-row: transforms per plane, banded solves of length n2)."""
    from oracle.lmvd import Config, Plan as OPlan, substep
    from paper_2206_09878_amd.workloads import make_inputs, workload
    w = workload(full.name, n=full.n1, n2=n2)
    inp = make_inputs(w, seed=2)
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    cfg = Config(w.n1, w.n3, w.n2, w.order, w.m1, w.m3, w.L1, w.L2, w.L3, w.breakpoints, w.dt, w.mu,
                 w.rhoD, w.g, w.rho_l, w.rho_h, w.beta_n, w.beta_p, w.kf, tuple(w.mu_z), tuple(w.rhoD_z),
                 w.rhoD_form)
    op = OPlan(cfg)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    substep(op, st, 0, hist=inp["hist"])
    t = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    ratio = full.n2 / w.n2
    return {"value": 1.0 / (t * ratio), "unit": "substeps/s", "cores": max(1, round(cpu / t)), "kind": "oracle",
            "sample": f"one oracle substep (stage n, k_f={w.kf}) of the {full.name} recipe at "
                      f"{w.n1}x{w.n2}x{w.n3} ({w.m1}x{w.m3} grid): {t:.1f} s wall, {cpu:.1f} s CPU; scaled "
                      f"linearly in n2 by {ratio:.2f} to {full.n1}x{full.n2}x{full.n3}"}


def main():
    names = class_names()
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rt512")
    ap.add_argument("--plane-batch", type=int, default=0)
    ap.add_argument("--transport", choices=["constant", "variable"], default="constant",
                    help="variable: mu(z) = mu (1 + z/2 - 0.3 z^2 + 0.2 z^3), rho D_z = f(z) rhoD (1 + 0.4 z + "
                         "0.1 z^2 - 0.05 z^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-class", choices=names, default=None,
                    help="time this kernel class instead of detecting the dominant one")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only copy a GIB-sized device buffer three times (reference kernel for the HBM "
                         "byte counters) and exit")
    ap.add_argument("--hbm-ceiling", type=float, default=0.0, metavar="GIB",
                    help="only time plain streaming kernels over GIB-sized buffers (the practical HBM "
                         "ceiling) and exit")
    args = ap.parse_args()
    if args.hbm_ceiling > 0:
        print(json.dumps(hbm_ceiling(args.hbm_ceiling)), flush=True)
        return
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2**30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": 8 * n, "dispatches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the substep runs on one GPU only; sharding across GPUs is designed, not implemented. "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2206_09878_amd.lmvd import Plan, Stepper
    from paper_2206_09878_amd.workloads import make_inputs, workload

    torch.cuda.set_device(0)
    if args.workload == "batch64":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "adjoint96":
        print(json.dumps(bench_adjoint(args)), flush=True)
        return
    w = workload(args.workload)
    if args.transport == "variable":
        w = dataclasses.replace(w, mu_z=(0.5 * w.mu, -0.3 * w.mu, 0.2 * w.mu),
                                rhoD_z=(0.4 * w.rhoD, 0.1 * w.rhoD, -0.05 * w.rhoD), rhoD_form=1)
    plan = Plan(w, plane_batch=args.plane_batch)
    stepper = Stepper(plan, make_inputs(w, seed=2, stage=0), stage=0)
    for _ in range(args.warmup):
        stepper.substep()
    torch.cuda.synchronize()

    # dominant kernel class: one untimed substep per class with its launches timed
    totals, tbytes = {}, {}
    if args.kernel_class is None:
        for cls in range(len(names)):
            if names[cls] == "xpass_io":
                continue
            plan.profile_start(cls)
            stepper.substep()
            ms, n, b = plan.profile_stop()
            totals[cls] = ms
            tbytes[cls] = b
        dom = max(totals, key=totals.get)
    else:
        dom = names.index(args.kernel_class)
    torch.cuda.synchronize()

    # timed region: the substeps alone, no timing hook
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stepper.substep()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # the dominant class in a pass of its own: the same number of substeps, its launches bracketed by
    # HIP events on the library's stream
    plan.profile_start(dom)
    for _ in range(args.steps):
        stepper.substep()
    kms, klaunch, kbytes = plan.profile_stop()
    torch.cuda.synchronize()

    value = args.steps / elapsed
    avg_ms = kms / max(klaunch, 1)
    mbytes = model_bytes_per_substep(names[dom], w, w.kf)
    alg_per_launch = mbytes * args.steps / max(klaunch, 1) if mbytes is not None else None
    comp_per_launch = kbytes / max(klaunch, 1)
    achieved = (alg_per_launch / (avg_ms * 1e-3) / 1e9) if alg_per_launch is not None else None
    traffic = counter_traffic(names[dom], w)
    model = substep_model_bytes(w, w.kf)
    out = {
        "metric": f"RK substeps/s at {w.n1}x{w.n2}x{w.n3} FP64",
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
        "config": {"workload": f"{w.name}: {KIND.get(w.name, 'synthetic fields')}, density ratio "
                               f"{w.rho_h / w.rho_l:.2f}, {w.n1}x{w.n2}x{w.n3} modes, {w.m1}x{w.m3} dealiased x-z "
                               f"grid, k_f={w.kf}, stages n/' alternating",
                   "kf": w.kf, "plane_batch": args.plane_batch or w.n2, "transport": args.transport},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved is not None else None,
                     "traffic": traffic,
                     "kernel_class": names[dom], "kernel": kernel_symbol(names[dom], w),
                     "launches": klaunch, "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": alg_per_launch,
                     "compulsory_bytes_per_launch": comp_per_launch,
                     "compulsory_frac": comp_per_launch / (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                     "traffic_over_algorithmic": (traffic / alg_per_launch) if traffic and alg_per_launch else None,
                     "share_of_substep": (totals[dom] / sum(totals.values())) if totals else None},
        "substep_roofline": {"model_bytes_per_substep": model,
                             "frac": model * value / (HBM_PEAK_GBS * 1e9)},
        "kernel_class_ms_per_substep": {names[c]: totals[c] for c in totals},
        "kernel_class_tbps": {names[c]: tbytes[c] / (totals[c] * 1e-3) / 1e12 for c in totals if totals[c] > 0},
        "compulsory_bytes_per_substep": sum(tbytes.values()) if tbytes else None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
