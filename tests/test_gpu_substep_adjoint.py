"""The adjoint of the substep through the library (lmvd_substep_adjoint and the autograd substep built on
it), against the oracle's adjoint and against directional derivatives of the native forward.

  * element by element against oracle/adjoint.py, on the same inputs and output cotangents: both
    stages, BDF and zero guesses, k_f = 4 and 1, density ratio 3 with gravity; 32 x 33 x 32 (register
    transform kernels) and 24 x 25 x 24 (generic kernels, ragged plane batches of 7);
  * the autograd substep (forward lmvd_substep, backward lmvd_substep_adjoint) against central
    differences of lmvd_substep;
  * the adjoint workload: 96 x 97 x 96, density 1 -> 7 layer, 20 RK steps with checkpointed
    recomputation every 5 steps, objective the domain-averaged kinetic energy |m|^2 / (2 rho) with
    m = m^d + m^c at the final time (Gauss-Legendre in y), its gradient with respect to the initial z
    against central differences (eps = 1e-6 relative, extrapolated from eps and eps/2) on 16 random
    directions; the times of the native forward and of the checkpointed forward + backward are
    printed."""
import numpy as np
import pytest

from oracle.adjoint import substep_adjoint as oracle_adjoint
from oracle.lmvd import Plan as OPlan
from paper_2206_09878_amd.workloads import make_inputs, workload
from tests.conftest import oracle_config
from tests.test_gpu_parity import TOL, rel, spread_tolerances  # noqa: F401

pytestmark = pytest.mark.gpu
STATE = ("phi2", "omega2", "z", "m1bar", "m3bar")
RHS = ("phi2", "omega2", "m1bar", "m3bar")


def herm(rng, shape, zero00=False):
    V = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nn = shape[1]
    for ni in range(1, (nn + 1) // 2):
        V[:, nn - ni, 0] = np.conj(V[:, ni, 0])
    V[:, 0, 0] = 0.0 if zero00 else V[:, 0, 0].real
    return V


def cotangents(w, seed):
    rng = np.random.default_rng(seed)
    S = lambda z=False: herm(rng, w.shape, z)
    v = lambda: rng.standard_normal(w.n2)
    return {"state": {"phi2": S(True), "omega2": S(True), "z": S(), "m1bar": v(), "m3bar": v()},
            "rhs": {"phi2": S(True), "omega2": S(True), "m1bar": v(), "m3bar": v()}, "zt": S(),
            "md": (S(), herm(rng, w.shape_star), S()), "mc": (S(), herm(rng, w.shape_star), S())}


def gpu_adjoint(w, stage, inp, cot, kf, guess_mode, plane_batch=0):
    import torch
    from paper_2206_09878_amd.lmvd import Plan
    p = Plan(w, plane_batch=plane_batch)
    d = lambda a: p.to_dev(a)
    inputs = {k: d(inp[k]) for k in STATE}
    inputs["hist"] = [d(h) for h in inp["hist"]]
    if stage == 1:
        inputs["rhs_prev"] = {k: d(v) for k, v in inp["rhs_prev"].items()}
        inputs["zt_prev"] = d(inp["zt_prev"])
    c = {k + "_out": d(cot["state"][k]) for k in STATE}
    c["rhs"] = {k: d(v) for k, v in cot["rhs"].items()}
    c["zt"] = d(cot["zt"])
    c["md"] = tuple(d(x) for x in cot["md"])
    c["mc"] = tuple(d(x) for x in cot["mc"])
    g = p.substep_adjoint(stage, inputs, c, kf=kf, guess_mode=guess_mode)
    torch.cuda.synchronize()
    h = lambda t: t.detach().cpu().numpy()
    out = {k: h(g[k]) for k in STATE}
    if guess_mode == 0:
        out["hist"] = [h(x) for x in g["hist"]]
    if stage == 1:
        out["rhs_prev"] = {k: h(v) for k, v in g["rhs_prev"].items()}
        out["zt_prev"] = h(g["zt_prev"])
    return out


def flat(g):
    out = {k: g[k] for k in STATE}
    for i, x in enumerate(g.get("hist") or []):
        out[f"hist{i}"] = x
    for k, v in (g.get("rhs_prev") or {}).items():
        out["rhs_prev_" + k] = v
    if g.get("zt_prev") is not None:
        out["zt_prev"] = g["zt_prev"]
    return out


CASES = [(32, 33, 0, 0, 4, 0), (32, 33, 1, 0, 4, 0), (32, 33, 0, 1, 1, 0), (24, 25, 1, 0, 4, 7),
         (24, 25, 0, 1, 4, 7), (16, 14, 1, 0, 4, 0), (16, 19, 0, 0, 4, 0)]  # the last two: other row counts


@pytest.mark.parametrize("n,n2,stage,guess_mode,kf,plane_batch", CASES)
def test_adjoint_against_the_oracle_adjoint(n, n2, stage, guess_mode, kf, plane_batch):
    import torch
    assert torch.cuda.is_available()
    w = workload("small", n=n, n2=n2)
    w.rho_l, w.rho_h, w.g = 1.0, 3.0, 1.0
    inp = make_inputs(w, seed=30 + n + stage, stage=stage)
    cot = cotangents(w, 50 + n + stage)
    op = OPlan(oracle_config(w))
    st = {k: inp[k] for k in STATE}
    guess = "zero" if guess_mode else "bdf"
    kw = dict(rhs_prev=inp.get("rhs_prev"), zt_prev=inp.get("zt_prev")) if stage == 1 else {}
    print(f"adjoint {n}x{n2}x{n} stage {stage} guess {guess} k_f {kf} plane batch {plane_batch or n2}", flush=True)
    ref = flat(oracle_adjoint(op, st, stage, cot, hist=inp["hist"], kf=kf, guess=guess, **kw))
    got = flat(gpu_adjoint(w, stage, inp, cot, kf, guess_mode, plane_batch))
    errs = {k: rel(got[k], ref[k]) for k in ref}
    print("  " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v < 1e-10}
    assert not bad, errs


def test_autograd_substep_matches_central_differences():
    """<grad_z L, v> of L = <W, outputs of one substep> through autograd.substep, against central
    differences of lmvd_substep (Richardson from eps and eps/2) on 4 random directions."""
    import torch
    from paper_2206_09878_amd.autograd import substep
    from paper_2206_09878_amd.lmvd import Plan
    w = workload("small")
    w.g = 1.0
    p = Plan(w)
    inp = make_inputs(w, seed=61, stage=0)
    st = {k: p.to_dev(inp[k]) for k in STATE}
    hist = [p.to_dev(h) for h in inp["hist"]]
    rng = np.random.default_rng(62)
    W = [p.to_dev(herm(rng, w.shape)) for _ in range(4)]

    def loss(z):
        r = substep(p, 0, dict(st, z=z), hist)
        outs = [r["state"]["phi2"], r["state"]["z"], r["rhs"]["omega2"], r["zt"]]
        return sum(torch.sum(torch.view_as_real(a) * torch.view_as_real(b)) for a, b in zip(outs, W))

    z0 = st["z"].clone().requires_grad_(True)
    loss(z0).backward()
    grad = z0.grad.detach()
    eps = 1e-6 * st["z"].abs().max().item()
    with torch.no_grad():
        for k in range(4):
            v = p.to_dev(herm(rng, w.shape))
            c = lambda e: (loss(st["z"] + e * v) - loss(st["z"] - e * v)).item() / (2 * e)
            fd = (4.0 * c(0.5 * eps) - c(eps)) / 3.0
            an = float(torch.sum(torch.view_as_real(grad) * torch.view_as_real(v)))
            print("direction", k, "extrapolated", fd, "adjoint", an, flush=True)
            assert abs(fd - an) < 1e-6 * max(abs(an), 1e-300), (k, fd, an)


def test_adjoint_workload_twenty_steps_checkpointed():
    import time

    import torch
    from paper_2206_09878_amd.adjoint import final_kinetic_energy, rollout
    from paper_2206_09878_amd.lmvd import Plan, Stepper
    w = workload("adjoint96")
    p = Plan(w)
    inp = make_inputs(w, seed=98, stage=0)
    st0 = {k: p.to_dev(inp[k]) for k in STATE}
    hist0 = [p.to_dev(h) for h in inp["hist"]]
    print("adjoint workload", (w.n1, w.n2, w.n3), "20 RK steps, checkpoint every 5", flush=True)

    # the native forward alone: 40 substeps on the plain path (Stepper), and the objective's substep
    s = Stepper(p, inp, stage=0)
    for _ in range(4):
        s.substep()
    s = Stepper(p, inp, stage=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(41):
        s.substep()
    torch.cuda.synchronize()
    t_native = time.perf_counter() - t0

    def objective(z0, ckpt):
        state, hist = rollout(p, dict(st0, z=z0), hist0, steps=20, checkpoint_every=5 if ckpt else None)
        return final_kinetic_energy(p, state, hist)

    with torch.no_grad():
        J = objective(st0["z"], False).item()
    z0 = st0["z"].clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    objective(z0, True).backward()
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    grad = z0.grad.detach()
    print(f"objective {J:.6e}; native forward {t_native:.3f} s, checkpointed forward + backward {t_adj:.3f} s, "
          f"ratio {t_adj / t_native:.1f}", flush=True)
    assert np.isfinite(J) and torch.isfinite(torch.view_as_real(grad)).all()
    eps = 1e-6 * st0["z"].abs().max().item()
    rng = np.random.default_rng(700)
    with torch.no_grad():
        for k in range(16):
            v = p.to_dev(herm(rng, w.shape))
            c = lambda e: (objective(st0["z"] + e * v, False) - objective(st0["z"] - e * v, False)).item() / (2 * e)
            f1, f2 = c(eps), c(0.5 * eps)
            fd = (4.0 * f2 - f1) / 3.0
            an = float(torch.sum(torch.view_as_real(grad) * torch.view_as_real(v)))
            print("direction", k, "central", f1, "extrapolated", fd, "adjoint", an, flush=True)
            assert abs(fd - an) < 1e-6 * max(abs(an), 1e-300), (k, f1, fd, an)
