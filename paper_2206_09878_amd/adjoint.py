"""Gradients through simulations: differentiable RK steps, checkpointed rollouts and the kinetic-energy
objective of the adjoint workload.

Every substep runs on the library (lmvd_substep forward, lmvd_substep_adjoint backward, through
autograd.substep); this module only strings substeps together as the two-stage RK2 scheme does (the z
history ring and the stored stage-n data) and defines the objective.

    from paper_2206_09878_amd.adjoint import rollout, final_kinetic_energy
    state, hist = rollout(plan, state0, hist0, steps=20, checkpoint_every=5)
    J = final_kinetic_energy(plan, state, hist)
    J.backward()                    # gradients in state0 / hist0 tensors that require them
"""
from __future__ import annotations

import numpy as np
import torch

from .autograd import substep
from .lmvd import basis_values

_STATE = ("phi2", "omega2", "z", "m1bar", "m3bar")


def rk_step(plan, state, hist, kf=-1):
    """One RK2 step (stage n, then stage ') from the state at t^n and its z history
    (z^{n-1,'}, z^{n-1}, z^{n-2,'}); returns the state at t^{n+1} and its history."""
    a = substep(plan, 0, state, hist, kf=kf)
    b = substep(plan, 1, a["state"], [state["z"], hist[0], hist[1]], prev=(a["rhs"], a["zt"]), kf=kf)
    return b["state"], [a["state"]["z"], state["z"], hist[0]]


def rollout(plan, state, hist, steps, checkpoint_every=None, kf=-1):
    """`steps` RK steps.  With checkpoint_every = c, the steps run in segments of c whose intermediate
    substeps are not kept for the backward pass: only each segment's input state is saved, and the
    segment is run again when its gradient is needed (torch.utils.checkpoint)."""
    if not checkpoint_every:
        for _ in range(steps):
            state, hist = rk_step(plan, state, hist, kf)
        return state, hist
    from torch.utils.checkpoint import checkpoint

    def segment(n, *flat):
        st, hs = dict(zip(_STATE, flat[:5])), list(flat[5:8])
        for _ in range(n):
            st, hs = rk_step(plan, st, hs, kf)
        return tuple(st[k] for k in _STATE) + tuple(hs)

    flat = tuple(state[k] for k in _STATE) + tuple(hist)
    done = 0
    while done < steps:
        n = min(checkpoint_every, steps - done)
        flat = checkpoint(segment, n, *flat, use_reentrant=False)
        done += n
    return dict(zip(_STATE, flat[:5])), list(flat[5:8])


def gauss_legendre_y(plan, per_interval=None):
    """Points and weights of the y quadrature: Gauss-Legendre with p + 1 points on every knot interval
    of the breakpoints (exact for polynomials of degree 2p + 1 on each interval)."""
    w = plan.w
    q = per_interval or (w.order + 1)
    x, wt = np.polynomial.legendre.leggauss(q)
    bp = np.asarray(w.breakpoints)
    ys, ws = [], []
    for a, b in zip(bp[:-1], bp[1:]):
        ys.append(0.5 * (b - a) * x + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wt)
    return np.concatenate(ys), np.concatenate(ws)


def _to_grid(plan, V):
    """Values [ny, N3-1, N1/2] (half spectrum) -> real field [ny, M3, M1] on the 3/2 grid."""
    w = plan.w
    ny, nn, nl = V.shape
    h = (nn + 1) // 2
    n = np.concatenate([np.arange(0, h), np.arange(-(h - 1), 0)]) % w.m3
    full = torch.zeros((ny, w.m3, w.m1 // 2 + 1), dtype=V.dtype, device=V.device)
    full = full.index_copy(1, torch.as_tensor(n, device=V.device),
                           torch.nn.functional.pad(V, (0, w.m1 // 2 + 1 - nl)))
    return torch.fft.irfft2(full, s=(w.m3, w.m1), norm="forward")


def kinetic_energy(plan, m1, m2, m3, z):
    """Domain average of |m|^2 / (2 rho), rho = f(z), from the B coefficients of m1, m3, z and the B*
    coefficients of m2: the x-z mean on the 3/2 grid, Gauss-Legendre in y (p + 1 points per knot
    interval).  Differentiable in all four (torch operations on the library's coefficient arrays)."""
    w = plan.w
    y, wy = gauss_legendre_y(plan)
    dev = z.device
    B = torch.as_tensor(basis_values(w, y), device=dev).to(torch.complex128)
    Bs = torch.as_tensor(basis_values(w, y, star=True), device=dev).to(torch.complex128)
    at = lambda M, c: torch.tensordot(M, c, dims=([1], [0]))
    zp = _to_grid(plan, at(B, z))
    rho = w.rho_l * w.rho_h / (w.rho_h - (w.rho_h - w.rho_l) * zp)
    ke = (_to_grid(plan, at(B, m1)) ** 2 + _to_grid(plan, at(Bs, m2)) ** 2 + _to_grid(plan, at(B, m3)) ** 2) / rho
    wy = torch.as_tensor(wy, device=dev)
    return 0.5 * torch.sum(wy * ke.mean(dim=(1, 2))) / w.L2


def final_kinetic_energy(plan, state, hist, kf=-1):
    """The kinetic-energy objective at the state's time: m = m^d + m^c with m^d from the state and m^c
    from the fixed point at that state (the m^c of a stage-n substep started there, which also gives
    m^d; its other outputs are not used)."""
    r = substep(plan, 0, state, hist, kf=kf, diag=True)
    md, mc = r["md"], r["mc"]
    return kinetic_energy(plan, md[0] + mc[0], md[1] + mc[1], md[2] + mc[2], state["z"])
