"""Single-mode Rayleigh-Taylor runs on the GPU path (Section 5 of the paper):
bubble and spike heights and the bubble velocity in the potential-growth
phase, against the closed form of Goncharov,

    v_b = sqrt( 2 At / (1 + At) * g / (C k) ),   C = 1 (3D), k = 2 pi / W.

Set-up as the paper's cases: horizontally periodic W x W box, x2 in [-2W, 2W]
(or [-3.5W, 3.5W] with the interface raised by 0.5W at high Atwood number),
heavy fluid on top, gravity along -x2, z = (1 + tanh((x2 - h) / (2 eps W))) / 2
with eps = 0.05 and, in 3D, h / W = 0.05 (cos(2 pi x1 / W) + cos(2 pi x3 / W)),
Re = 1024; in 2D, h / W = 0.1 cos(2 pi x1 / W), Re = 3000 (the x3 direction
is kept with a field independent of x3, which the substep preserves exactly).
Sc = 1 (rho D = mu), Re = rho_h sqrt(W^3 g) / mu, and an initial momentum that
is the curl-free diffusion flux (m^d = 0).  Goncharov's constant is C = 1 in
3D and C = 3 in 2D.

Everything runs through the library: the initial z is formed on the 3/2 grid
at the Greville points, brought to spectral values by lmvd_to_spectral and to
B coefficients by lmvd_project; heights come from lmvd_evaluate and
lmvd_to_physical.

    python -m paper_2206_09878_amd.validate_rt [--at 0.5] [--dim 3] [--n 32] [--n3 N] [--n2 257] [--dt 1e-3] [--tau 3]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from .workloads import Workload


def goncharov_vb(at: float, g: float = 1.0, w: float = 1.0, dim: int = 3) -> float:
    c = 1.0 if dim == 3 else 3.0
    return math.sqrt(2.0 * at / (1.0 + at) * g / (c * 2.0 * math.pi / w))


def rt_workload(at: float, n: int, n2: int, dt: float, re: float | None = None, kf: int = 4, dim: int = 3,
                n3: int | None = None) -> Workload:
    """The paper's box: x2 in [-2W, 2W] with the interface at 0 for the lower Atwood numbers,
    [-3.5W, 3.5W] with the interface raised by delta = 0.5W for the higher ones.  n3 (default n) sets
    the x3 modes; in 2D the fields do not depend on x3."""
    rho_h = 1.0
    rho_l = rho_h * (1.0 - at) / (1.0 + at)
    re = (1024.0 if dim == 3 else 3000.0) if re is None else re
    mu = rho_h / re  # W = g = 1
    high = at > 0.7
    n3 = n if n3 is None else n3
    return Workload(f"rt_single_{dim}d_at{at}", n, n3, n2, 3 * n // 2, 3 * n3 // 2, 1.0, 7.0 if high else 4.0,
                    1.0, 1.0, dt=dt, mu=mu, rhoD=mu, g=1.0, rho_l=rho_l, rho_h=rho_h, kf=kf,
                    extra=dict(eps=0.05, amp=0.05 if dim == 3 else 0.1, delta=0.5 if high else 0.0, dim=dim))


def plateau_velocity(r: dict, lo: float = 1.3, hi: float = 2.5) -> float:
    """Least-squares slope of h_b(t) over tau in [lo, hi] (the near-constant phase), in units of sqrt(W g)."""
    t = np.asarray(r["tau"])
    hb = np.asarray(r["h_b"])
    m = (t >= lo) & (t <= hi) & np.isfinite(hb)
    return float(np.polyfit(t[m] / math.sqrt(r["at"]), hb[m], 1)[0])


def crossing(y: np.ndarray, f: np.ndarray, level: float = 0.5) -> float:
    """Height where f (increasing upward through the interface) crosses level, by
    linear interpolation between the sample heights; the crossing nearest the
    middle of the largest jump."""
    s = f - level
    idx = np.nonzero((s[:-1] <= 0) & (s[1:] > 0))[0]
    if idx.size == 0:
        return float("nan")
    j = idx[np.argmax(f[idx + 1] - f[idx])]
    return float(y[j] + (y[j + 1] - y[j]) * (level - f[j]) / (f[j + 1] - f[j]))


def run(at: float = 0.5, n: int = 32, n2: int = 257, dt: float = 1e-3, tau_end: float = 3.0,
        every: int = 10, re: float | None = None, verbose: bool = False, dim: int = 3, n3: int | None = None) -> dict:
    import torch

    from .lmvd import Plan, Stepper, host_tables

    w = rt_workload(at, n, n2, dt, re, dim=dim, n3=n3)
    plan = Plan(w)
    tau_pts, _, _ = host_tables(w)
    eps, amp = w.extra["eps"], w.extra["amp"]
    x1 = np.arange(w.m1) * w.L1 / w.m1
    x3 = np.arange(w.m3) * w.L3 / w.m3
    c3 = np.cos(2 * math.pi * x3) if dim == 3 else np.zeros_like(x3)
    h = amp * (c3[:, None] + np.cos(2 * math.pi * x1)[None, :]) + w.extra["delta"]
    zphys = 0.5 * (1.0 + np.tanh((tau_pts[:, None, None] - h[None]) / (2.0 * eps)))
    vals = plan.to_spectral(torch.from_numpy(np.ascontiguousarray(zphys)).cuda())
    zc = plan.project(0, vals)
    torch.cuda.synchronize()
    z0 = zc.cpu().numpy()
    zero = np.zeros(w.shape, dtype=np.complex128)
    inputs = dict(phi2=zero, omega2=zero.copy(), z=z0, m1bar=np.zeros(w.n2), m3bar=np.zeros(w.n2),
                  hist=[z0, z0, z0])
    st = Stepper(plan, inputs, stage=0)

    def heights():
        phys = plan.to_physical(plan.evaluate(0, st.z)).cpu().numpy()
        return (crossing(tau_pts, phys[:, 0, 0]), crossing(tau_pts, phys[:, w.m3 // 2, w.m1 // 2]))

    sq = math.sqrt(at)  # time unit of the figures: tau = t sqrt(At g / W)
    t, rows = 0.0, []
    hb, hs = heights()
    rows.append((0.0, hb, hs))
    nsteps = int(math.ceil(tau_end / sq / dt))
    t0 = time.perf_counter()
    for k in range(1, nsteps + 1):
        st.substep()
        st.substep()
        t += dt
        if k % every == 0 or k == nsteps:
            hb, hs = heights()
            rows.append((t * sq, hb, hs))
            if not (np.isfinite(hb) and np.isfinite(hs)):
                break
        if verbose and k % 500 == 0:
            print(f"step {k}/{nsteps}  tau {t * sq:.3f}  h_b {hb:.4f}  h_s {hs:.4f}", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    a = np.array(rows)
    tt, hbs = a[:, 0], a[:, 1]
    vb = np.gradient(hbs, tt / sq)  # d h_b / dt in units of sqrt(W g)
    return {"at": at, "dim": dim, "grid": [w.n1, w.n2, w.n3], "dt": dt, "re": w.rho_h / w.mu, "steps": k,
            "wall_s": wall, "tau": tt.tolist(), "h_b": hbs.tolist(), "h_s": a[:, 2].tolist(), "v_b": vb.tolist(),
            "v_b_goncharov": goncharov_vb(at, dim=dim)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--at", type=float, default=0.5)
    ap.add_argument("--dim", type=int, choices=[2, 3], default=3)
    ap.add_argument("--n3", type=int, default=None)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--n2", type=int, default=257)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--tau", type=float, default=3.0)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    r = run(a.at, a.n, a.n2, a.dt, a.tau, a.every, verbose=True, dim=a.dim, n3=a.n3)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(r, f)
    vb = np.array(r["v_b"])
    print(json.dumps({"at": r["at"], "dim": r["dim"], "grid": r["grid"], "dt": r["dt"], "steps": r["steps"],
                      "wall_s": round(r["wall_s"], 1), "v_b_max": float(np.nanmax(vb)),
                      "v_b_plateau": plateau_velocity(r), "v_b_goncharov": r["v_b_goncharov"]}), flush=True)


if __name__ == "__main__":
    main()
