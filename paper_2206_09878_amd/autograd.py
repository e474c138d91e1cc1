"""Automatic differentiation through the linear building blocks of the substep.

Each operator is a torch.autograd.Function whose forward is the library's
operator and whose backward is its transpose (lmvd_*_adjoint), so gradients of
real losses follow PyTorch's convention for complex inputs (dL/dRe + i dL/dIm).

    from paper_2206_09878_amd.autograd import to_physical, to_spectral, evaluate, project, md, mc
    loss = (to_physical(plan, evaluate(plan, 0, project(plan, 0, v))) * w).sum()
    loss.backward()          # v.grad through P^T, E_0^T and the transposed transform

The operators are linear, so their backward needs no saved state.
"""
from __future__ import annotations

import torch


class _ToPhysical(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, values):
        ctx.plan = plan
        return plan.to_physical(values.contiguous())

    @staticmethod
    def backward(ctx, g):
        return None, ctx.plan.to_physical_adjoint(g.contiguous())


class _ToSpectral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, phys):
        ctx.plan = plan
        return plan.to_spectral(phys.contiguous())

    @staticmethod
    def backward(ctx, g):
        return None, ctx.plan.to_spectral_adjoint(g.contiguous())


class _Mc(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, rhot):
        ctx.plan = plan
        return plan.mc(rhot.contiguous())

    @staticmethod
    def backward(ctx, g1, g2, g3):
        z = lambda g, star: g.contiguous() if g is not None else ctx.plan.empty(star).zero_()
        return None, ctx.plan.mc_adjoint(z(g1, False), z(g2, True), z(g3, False))


class _Md(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, phi2, omega2, m1bar, m3bar):
        ctx.plan = plan
        return plan.md(phi2.contiguous(), omega2.contiguous(), m1bar.contiguous(), m3bar.contiguous())

    @staticmethod
    def backward(ctx, g1, g2, g3):
        z = lambda g, star: g.contiguous() if g is not None else ctx.plan.empty(star).zero_()
        tp, to, t1, t3 = ctx.plan.md_adjoint(z(g1, False), z(g2, True), z(g3, False))
        return None, tp, to, t1, t3


class _Evaluate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, deriv, star, coeffs):
        ctx.plan, ctx.deriv, ctx.star = plan, deriv, star
        return plan.evaluate(deriv, coeffs.contiguous(), star=star)

    @staticmethod
    def backward(ctx, g):
        return None, None, None, ctx.plan.evaluate_adjoint(ctx.deriv, g.contiguous(), star=ctx.star)


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, kind, values):
        ctx.plan, ctx.kind = plan, kind
        return plan.project(kind, values.contiguous())

    @staticmethod
    def backward(ctx, g):
        return None, None, ctx.plan.project_adjoint(ctx.kind, g.contiguous())


def to_physical(plan, values):
    """Values at the Greville points (S-field) -> physical field on the 3/2 grid, differentiable."""
    return _ToPhysical.apply(plan, values)


def to_spectral(plan, phys):
    """Physical field on the 3/2 grid -> values at the Greville points (S-field), differentiable."""
    return _ToSpectral.apply(plan, phys)


def md(plan, phi2, omega2, m1bar, m3bar):
    """m^d = (m1, m2 in B*, m3) from (phi2, Omega2, <m>1, <m>3), differentiable."""
    return _Md.apply(plan, phi2, omega2, m1bar, m3bar)


def mc(plan, rhot):
    """m^c = (m1, m2 in B*, m3) from the B coefficients of rho_t, differentiable."""
    return _Mc.apply(plan, rhot)


def evaluate(plan, deriv, coeffs, star=False):
    """E_deriv (or F_0 with star) applied to B (B*) coefficients, differentiable."""
    return _Evaluate.apply(plan, deriv, star, coeffs)


def project(plan, kind, values):
    """Values -> coefficients (kind 0 plain, 1 Dirichlet, 2 Neumann rows), differentiable."""
    return _Project.apply(plan, kind, values)


# ---------------------------------------------------------------------------
# the whole substep

_STATE = ("phi2", "omega2", "z", "m1bar", "m3bar")
_RHS = ("phi2", "omega2", "m1bar", "m3bar")


class _Substep(torch.autograd.Function):
    """Forward: lmvd_substep.  Backward: lmvd_substep_adjoint, which recomputes the substep's
    intermediates from the saved inputs (the state, the z history and, at stage ', the stage-n data)."""

    @staticmethod
    def forward(ctx, plan, stage, kf, guess_mode, diag, phi2, omega2, z, m1bar, m3bar, h0, h1, h2,
                rp_phi2, rp_omega2, rp_m1, rp_m3, zt_prev):
        ctx.plan, ctx.stage, ctx.kf, ctx.guess_mode, ctx.diag = plan, stage, kf, guess_mode, diag
        hist = [h0, h1, h2] if guess_mode == 0 else None
        ins = [phi2, omega2, z, m1bar, m3bar] + (hist or [None] * 3)
        rp = dict(zip(_RHS, (rp_phi2, rp_omega2, rp_m1, rp_m3))) if stage == 1 else None
        ins += list(rp.values()) + [zt_prev] if stage == 1 else [None] * 5
        ctx.save_for_backward(*ins)
        c = lambda t: t.contiguous()
        vec = lambda: torch.empty(plan.w.n2, dtype=torch.float64, device="cuda")
        out = {"phi2": plan.empty(), "omega2": plan.empty(), "z": plan.empty(), "m1bar": vec(), "m3bar": vec()}
        rhs = {"phi2": plan.empty(), "omega2": plan.empty(), "m1bar": vec(), "m3bar": vec()}
        zt = plan.empty()
        md = [plan.empty(), plan.empty(True), plan.empty()] if diag else None
        mc = [plan.empty(), plan.empty(True), plan.empty()] if diag else None
        plan.substep(stage, c(phi2), c(omega2), c(z), c(m1bar), c(m3bar), z_out=out["z"], phi2_out=out["phi2"],
                     omega2_out=out["omega2"], m1bar_out=out["m1bar"], m3bar_out=out["m3bar"],
                     hist=[c(h) for h in hist] if hist else None, kf=kf, guess_mode=guess_mode,
                     rhs_prev={k: c(v) for k, v in rp.items()} if rp else None,
                     zt_prev=c(zt_prev) if stage == 1 else None, rhs_out=rhs, zt_out=zt, md=md, mc=mc)
        res = [out[k] for k in _STATE] + [rhs[k] for k in _RHS] + [zt]
        if diag:
            res += md + mc
        return tuple(res)

    @staticmethod
    def backward(ctx, *g):
        plan = ctx.plan
        saved = ctx.saved_tensors
        inputs = dict(zip(_STATE, saved[:5]))
        if ctx.guess_mode == 0:
            inputs["hist"] = list(saved[5:8])
        if ctx.stage == 1:
            inputs["rhs_prev"] = dict(zip(_RHS, saved[8:12]))
            inputs["zt_prev"] = saved[12]
        cot = {k + "_out": g[i] for i, k in enumerate(_STATE)}
        cot["rhs"] = {k: g[5 + i] for i, k in enumerate(_RHS)}
        cot["zt"] = g[9]
        if ctx.diag:
            cot["md"] = tuple(g[10:13])
            cot["mc"] = tuple(g[13:16])
        gr = plan.substep_adjoint(ctx.stage, inputs, cot, kf=ctx.kf, guess_mode=ctx.guess_mode)
        hist_g = gr.get("hist") or [None] * 3
        prev_g = [gr["rhs_prev"][k] for k in _RHS] + [gr["zt_prev"]] if ctx.stage == 1 else [None] * 5
        return (None, None, None, None, None, *[gr[k] for k in _STATE], *hist_g, *prev_g)


def substep(plan, stage, state, hist=None, prev=None, kf=-1, guess_mode=0, diag=False):
    """One differentiable substep (Algorithm time_advanceDNS) through the library.

    state: dict phi2, omega2, z, m1bar, m3bar (device tensors); hist: the z history (3 tensors, most
    recent first) for the BDF-like guess; prev: at stage ', (RHS dict, z_t) of stage n.  Returns a dict:
    state (new), rhs, zt and, with diag, md and mc (m2 in B*).  Gradients flow to every tensor input."""
    rp = prev[0] if prev is not None else {}
    zt_prev = prev[1] if prev is not None else None
    h = list(hist) if hist is not None else [None] * 3
    out = _Substep.apply(plan, stage, kf, guess_mode, diag, *[state[k] for k in _STATE], *h,
                         *[rp.get(k) for k in _RHS], zt_prev)
    res = {"state": dict(zip(_STATE, out[:5])), "rhs": dict(zip(_RHS, out[5:9])), "zt": out[9]}
    if diag:
        res["md"], res["mc"] = tuple(out[10:13]), tuple(out[13:16])
    return res
