"""Pins of the oracle's adjoint substep (oracle/adjoint.py) against the forward oracle, by routes other
than its own formulas:

  * every transpose satisfies <A x, y> = <x, A^T y> against its forward operator (the inverse and
    forward transforms, the three projections, m^d, m^c), on random inputs the library accepts;
  * the whole substep: for random directions v over all inputs and random cotangents w over all
    outputs, <v, J^T w> from the adjoint equals <J v, w> with J v from central differences of the
    forward oracle (Richardson-extrapolated from steps h and h/2, per group of inputs; the difference
    falls as h^4 to the adjoint's value), for both stages, the BDF and the
    zero guess and k_f = 0, 1, 2, on a 12 x 13 x 12 grid at density ratio 3 with gravity.

A mistake in any transpose, a dropped Jacobian term, a wrong sign or a missing path fails the second
pin by many orders of magnitude more than its bar.  (The bulk-viscosity term -2/3 mu theta delta_ij
reaches no output, so its transpose cannot be pinned this way; it is kept as the forward has it.)"""
import numpy as np
import pytest

from oracle.adjoint import md_t, mc_t, project_t, substep_adjoint, to_physical_t, to_spectral_t
from oracle.fourier import to_physical, to_spectral
from oracle.lmvd import Plan, curl_free_momentum, divergence_free_momentum, substep
from paper_2206_09878_amd.workloads import make_inputs, workload
from tests.conftest import oracle_config


def rdot(a, b):
    return float(np.sum((np.conj(np.asarray(a)) * np.asarray(b)).real))


def herm(rng, shape, zero00=False):
    V = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nn = shape[1]
    for ni in range(1, (nn + 1) // 2):
        V[:, nn - ni, 0] = np.conj(V[:, ni, 0])
    V[:, 0, 0] = 0.0 if zero00 else V[:, 0, 0].real
    return V


def small_plan(n=12, n2=13, ratio=3.0):
    """12 x 13 x 12 with density ratio 3 and gravity on (so that the buoyancy term has a transpose to
    check)."""
    w = workload("small", n=n, n2=n2)
    w.rho_l, w.rho_h, w.g = 1.0, ratio, 1.0
    return Plan(oracle_config(w)), w


def test_linear_transposes():
    plan, w = small_plan()
    rng = np.random.default_rng(1)
    c = plan.cfg
    V = herm(rng, w.shape)
    u = rng.standard_normal((w.n2, w.m3, w.m1))
    assert abs(rdot(to_physical(V, c.m1, c.m3), u) - rdot(V, to_physical_t(plan, u))) < 1e-10 * abs(rdot(V, V))
    for Y in (herm(rng, w.shape), rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)):
        assert abs(rdot(to_spectral(u, c.n1, c.n3), Y) - rdot(u, to_spectral_t(plan, Y))) < 1e-12 * np.abs(u).sum()
    for kind in ("plain", "dirichlet", "neumann"):
        X, Y = herm(rng, w.shape), herm(rng, w.shape)
        lhs = rdot(plan.project(X, kind), Y)
        assert abs(lhs - rdot(X, project_t(plan, Y, kind))) < 1e-11 * np.abs(lhs + 1)
    # m^d: (phi2, Omega2, <m>1, <m>3) -> (m1, m2 in B*, m3)
    phi, om = herm(rng, w.shape, True), herm(rng, w.shape, True)
    mb1, mb3 = rng.standard_normal(w.n2), rng.standard_normal(w.n2)
    out = divergence_free_momentum(plan, phi, om, mb1, mb3)
    cot = (herm(rng, w.shape), herm(rng, w.shape_star), herm(rng, w.shape))
    lhs = sum(rdot(o, y) for o, y in zip(out, cot))
    g = md_t(plan, *cot)
    rhs = rdot(phi, g[0]) + rdot(om, g[1]) + rdot(mb1, g[2]) + rdot(mb3, g[3])
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    # m^c: rho_t -> (m1, m2 in B*, m3)
    rt = herm(rng, w.shape)
    out = curl_free_momentum(plan, rt)[:3]
    cot = (herm(rng, w.shape), herm(rng, w.shape_star), herm(rng, w.shape))
    lhs = sum(rdot(o, y) for o, y in zip(out, cot))
    assert abs(lhs - rdot(rt, mc_t(plan, *cot))) < 1e-10 * abs(lhs)


STATE = ("phi2", "omega2", "z", "m1bar", "m3bar")


def flat_outputs(res):
    """The substep's outputs as one list: state, RHS, z_t, m^d, m^c."""
    out = [res["state"][k] for k in STATE] + [res["rhs"][k] for k in ("phi2", "omega2", "m1bar", "m3bar")]
    return out + [res["zt"]] + list(res["diag"]["md"]) + list(res["diag"]["mc"])


@pytest.mark.parametrize("stage,guess,kf", [(0, "bdf", 2), (1, "bdf", 1), (0, "zero", 0), (1, "zero", 2)])
def test_adjoint_matches_directional_derivatives(stage, guess, kf):
    plan, w = small_plan()
    rng = np.random.default_rng(10 + stage + 3 * kf)
    inp = make_inputs(w, seed=5, stage=stage)
    st = {k: inp[k] for k in STATE}
    hist = inp["hist"]
    rp = inp.get("rhs_prev")
    zp = inp.get("zt_prev")

    def run(st_, hist_, rp_, zp_):
        kw = dict(rhs_prev=rp_, zt_prev=zp_) if stage == 1 else {}
        return substep(plan, st_, stage, hist=hist_, kf=kf, guess=guess, diagnostics=True, **kw)

    ref = run(st, hist, rp, zp)
    # cotangents of every output and directions over every input (the library's input contract)
    outs = flat_outputs(ref)
    W = [herm(rng, o.shape) if np.iscomplexobj(o) else rng.standard_normal(o.shape) for o in outs]
    cot = {"state": dict(zip(STATE, W[:5])), "rhs": dict(zip(("phi2", "omega2", "m1bar", "m3bar"), W[5:9])),
           "zt": W[9], "md": tuple(W[10:13]), "mc": tuple(W[13:16])}
    g = substep_adjoint(plan, st, stage, cot, hist=hist, rhs_prev=rp, zt_prev=zp, kf=kf, guess=guess)

    def scaled(x):
        return np.abs(x).max()

    V = {"phi2": herm(rng, w.shape, True) * scaled(st["phi2"]), "omega2": herm(rng, w.shape, True) * scaled(st["omega2"]),
         "z": herm(rng, w.shape) * 0.05, "m1bar": rng.standard_normal(w.n2) * 0.05,
         "m3bar": rng.standard_normal(w.n2) * 0.05}
    Vh = [herm(rng, w.shape) * 0.05 * w.dt for _ in range(3)]
    Vrp = {"phi2": herm(rng, w.shape, True), "omega2": herm(rng, w.shape, True),
           "m1bar": rng.standard_normal(w.n2), "m3bar": rng.standard_normal(w.n2)} if stage == 1 else None
    Vzp = herm(rng, w.shape) * 0.05 if stage == 1 else None

    zero = lambda d: {k: 0 * v for k, v in d.items()} if isinstance(d, dict) else (
        [0 * x for x in d] if isinstance(d, list) else (None if d is None else 0 * d))
    # each group of inputs with its own step: the state (z enters the guess with 1/dt, so the map is
    # strongly curved in z and the step is small), the history and the stage-n data (they enter
    # linearly, so a large step keeps the differencing clear of rounding)
    groups = [("state", 3e-5, (V, zero(Vh), zero(Vrp), zero(Vzp)))]
    if guess == "bdf":
        groups.append(("hist", 1.0, (zero(V), Vh, zero(Vrp), zero(Vzp))))
    if stage == 1:
        groups.append(("stage-n data", 1.0, (zero(V), zero(Vh), Vrp, zero(Vzp))))
        groups.append(("z_t^n", 1.0, (zero(V), zero(Vh), zero(Vrp), Vzp)))
    for name, h, (V_, Vh_, Vrp_, Vzp_) in groups:
        def J(hh):
            def at(s):
                st_ = {k: st[k] + s * hh * V_[k] for k in STATE}
                hist_ = [x + s * hh * v for x, v in zip(hist, Vh_)] if guess == "bdf" else hist
                rp_ = {k: rp[k] + s * hh * Vrp_[k] for k in rp} if stage == 1 else None
                zp_ = zp + s * hh * Vzp_ if stage == 1 else None
                return sum(rdot(o, y) for o, y in zip(flat_outputs(run(st_, hist_, rp_, zp_)), W))
            return (at(1.0) - at(-1.0)) / (2 * hh)

        fd = (4.0 * J(h / 2) - J(h)) / 3.0
        an = sum(rdot(V_[k], g[k]) for k in STATE)
        if guess == "bdf":
            an += sum(rdot(v, gh) for v, gh in zip(Vh_, g["hist"]))
        if stage == 1:
            an += sum(rdot(Vrp_[k], g["rhs_prev"][k]) for k in Vrp_) + rdot(Vzp_, g["zt_prev"])
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an)), (name, fd, an)
