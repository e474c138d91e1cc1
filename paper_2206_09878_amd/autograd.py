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
