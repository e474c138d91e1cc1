"""Scalar model of the temporal scheme (Section 3.3, system ODE, Algorithm
time_advanceODE) and the linear test problem of the stability analysis.

TEST INFRASTRUCTURE ONLY (pins of the time discretisation used by the oracle
substep; never imported by the product path).

Model (temporal convergence test of Section 3.3.1):
    dz/dt   = M1(z) dz/dt + M2(z),  M1 = c1 (1 + sin z), M2 = c2 exp(z)
    dmd/dt  = M3(md, mc) = c3 md mc^3
    drho/dt = G(mc) = c4 mc,        rho = f(z) = z
with c1 = .6i, c2 = -1, c3 = 2 - .8i, c4 = -3 + .5i, z0 = md0 = .5.
"""
from __future__ import annotations

import numpy as np

from .lmvd import bdf_coefficients

C1, C2, C3, C4 = 0.6j, -1.0 + 0j, 2.0 - 0.8j, -3.0 + 0.5j


def M1(z):
    return C1 * (1.0 + np.sin(z))


def M2(z):
    return C2 * np.exp(z)


def M3(md, mc):
    return C3 * md * mc ** 3


def exact_rhs(t, y):
    """Reduced system with I - M1 inverted exactly (the reference)."""
    z, md = y[0] + 1j * y[1], y[2] + 1j * y[3]
    zt = M2(z) / (1.0 - M1(z))
    mc = zt / C4            # G^{-1}(f'(z) z_t), f' = 1
    mdt = M3(md, mc)
    return [zt.real, zt.imag, mdt.real, mdt.imag]


def fixed_point(z, guess, k):
    """k applications of z_t <- M1(z) z_t + M2(z) starting from the guess."""
    zt = guess
    for _ in range(k):
        zt = M1(z) * zt + M2(z)
    return zt


def integrate(dt, t_end, kf=4, k_startup=400, beta_n=0.0, beta_p=-4.0, z0=0.5, md0=0.5):
    """Advance the model with the paper's scheme to t_end; returns (z, md).

    Stage data follow the DNS substep: at each stage the fixed point is
    solved for the current state (guess from the z history, eq. dzdt_guesses),
    m^c = G^{-1}(f' z_t), and the state is advanced with explicit midpoint RK2.
    The first step has no history: zero guess and k_startup iterations.
    """
    nsteps = int(round(t_end / dt))
    z, md = complex(z0), complex(md0)
    hist = None
    for n in range(nsteps):
        startup = hist is None
        # stage n
        g = 0.0 if startup else sum(a * h for a, h in zip(
            bdf_coefficients(0, beta_n, beta_p), [z] + hist)) / dt
        zt_n = fixed_point(z, g, k_startup if startup else kf)
        mc = zt_n / C4
        R_n = M3(md, mc)
        zp, mdp = z + 0.5 * dt * zt_n, md + 0.5 * dt * R_n
        hist_p = [z] + (hist[:2] if hist else [z, z])
        # stage '
        g = 0.0 if startup else sum(a * h for a, h in zip(
            bdf_coefficients(1, beta_n, beta_p), [zp] + hist_p)) / dt
        zt_p = fixed_point(zp, g, k_startup if startup else kf)
        mc = zt_p / C4
        R_p = M3(mdp, mc)
        z_new = zp + dt * (zt_p - 0.5 * zt_n)
        md_new = mdp + dt * (R_p - 0.5 * R_n)
        hist = [zp, z, hist_p[1]]
        z, md = z_new, md_new
    return z, md


def linear_step_matrix(lam1, lam2dt, k, beta_p=-4.0):
    """Amplification matrix of one full step of the scheme on
    dz/dt = lam1 dz/dt + lam2 z (Section 3.3.2), built by applying the scheme
    to the unit history vectors [z^n, z^{n-1,'}, z^{n-1}, z^{n-2,'}]
    (beta^n = 0).  lam2dt = lam2 * dt; dt = 1 without loss of generality."""
    A = np.zeros((4, 4), dtype=complex)
    for col in range(4):
        hvec = np.zeros(4, dtype=complex)
        hvec[col] = 1.0
        z, h1, h2, h3 = hvec
        # iterate zt <- lam1 zt + lam2 z, k times, from the BDF guess (dt = 1)
        a = bdf_coefficients(0, 0.0, beta_p)
        zt = a[0] * z + a[1] * h1 + a[2] * h2 + a[3] * h3
        for _ in range(k):
            zt = lam1 * zt + lam2dt * z
        zt_n = zt
        zp = z + 0.5 * zt_n
        a = bdf_coefficients(1, 0.0, beta_p)
        zt = a[0] * zp + a[1] * z + a[2] * h1 + a[3] * h2
        for _ in range(k):
            zt = lam1 * zt + lam2dt * zp
        z_new = zp + (zt - 0.5 * zt_n)
        A[:, col] = [z_new, zp, z, h1]
    return A
