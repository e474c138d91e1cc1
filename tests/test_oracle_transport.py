"""Pins of the oracle's variable transport coefficients, mu = g(z) and
rho D_z (Section 2: the transport coefficients are known functions of z),
against closed forms computed another way:

  * the mean scalar equation with rho D = q(z) and with rho D = f(z) q(z):
    R_z = d/dy(rho D(z) z') / rho, the flux differentiated by a fine central
    difference (no chain rule);
  * an x-dependent z at constant density: the Fourier coefficients of
    div(q(z) grad z) / rho taken by a fine-grid FFT of the analytic field
    (the |grad z|^2 term has an x-part);
  * a mean shear u1(y) with mu(z(y)): RHS of <m>1 = (mu(z) u1')' by
    polynomial algebra;
  * one (l, n) mode of m2 with mu linear in z(y) and rho = f(z(y)) (so that
    div u != 0): RHS_phi2 = -k^2 N2 -
    d/dy(i k1 N1 + i k3 N3) with T_ij = mu (d_j u_i + d_i u_j - 2/3 theta
    delta_ij) formed by polynomial algebra (eqs. phi and the stress tensor).
"""
import numpy as np

from oracle.lmvd import apply
from tests.test_oracle_substep import P, interp, make_plan, robin_poly, run, zero_state


def _rz_mean(plan, z0):
    st = zero_state(plan)
    st["z"][:, 0, 0] = interp(plan, z0)
    out = run(plan, st, kf=1)
    return apply(plan.sp.E[0], out["diag"]["Rz"])[1:-1, 0, 0]


def test_variable_diffusivity_mean_scalar_equation():
    """z0(y) only, no momentum: R_z = (rho D(z0) z0')' / f(z0), both forms of rho D."""
    rl, rh = 1.0, 5.0
    z0 = P([0.5, 0.1, 0.0, -0.003])
    coef = (0.02, -0.01, 0.004)
    for form in (0, 1):
        plan, w = make_plan(rl, rh, rhoD=3e-3, rhoD_z=coef, rhoD_form=form)
        tau = plan.sp.tau[1:-1]
        f = lambda z: rl * rh / (rh - (rh - rl) * z)
        q = lambda z: 3e-3 + coef[0] * z + coef[1] * z ** 2 + coef[2] * z ** 3
        K = (lambda z: q(z)) if form == 0 else (lambda z: f(z) * q(z))
        flux = lambda y: K(z0(y)) * z0.deriv()(y)
        h = 1e-4
        exact = (flux(tau + h) - flux(tau - h)) / (2 * h) / f(z0(tau))
        got = _rz_mean(plan, z0)
        assert np.abs(got - exact).max() < 1e-8 * np.abs(exact).max(), form
        # the variable part matters: a constant rho D = q(z) at the mean differs
        plan0, _ = make_plan(rl, rh, rhoD=3e-3)
        assert np.abs(_rz_mean(plan0, z0) - exact).max() > 1e-3 * np.abs(exact).max()


def test_variable_diffusivity_with_an_x_mode():
    """Constant density rho0, z = z0(y) + eps s(y) cos(k x), q(z) = a + b z:
    R_z = div(q(z) grad z) / rho0, whose modes l = 0, 1, 2 come from the
    analytic field on a fine x grid."""
    rho0 = 1.5
    a, b = 2e-3, 0.03
    plan, w = make_plan(rho0, rho0, rhoD=a, rhoD_z=(b, 0.0, 0.0))
    z0, s, eps = P([0.5, 0.1]), P([1.0, 0.0, 0.2]), 0.05
    l = 1
    kx = 2 * np.pi * l / plan.cfg.L1
    st = zero_state(plan)
    st["z"][:, 0, 0] = interp(plan, z0)
    st["z"][:, 0, l] = 0.5 * eps * interp(plan, s)        # cos = (e^{ikx} + e^{-ikx}) / 2
    out = run(plan, st, kf=1)
    Rz = apply(plan.sp.E[0], out["diag"]["Rz"])
    tau = plan.sp.tau[1:-1]
    x = np.arange(64) * plan.cfg.L1 / 64
    Y, X = np.meshgrid(tau, x, indexing="ij")
    c, sn = np.cos(kx * X), np.sin(kx * X)
    z = z0(Y) + eps * s(Y) * c
    zx = -eps * kx * s(Y) * sn
    zy = z0.deriv()(Y) + eps * s.deriv()(Y) * c
    zxx = -eps * kx * kx * s(Y) * c
    zyy = z0.deriv(2)(Y) + eps * s.deriv(2)(Y) * c
    field = ((a + b * z) * (zxx + zyy) + b * (zx * zx + zy * zy)) / rho0
    modes = np.fft.fft(field, axis=1) / 64
    for m in (0, 1, 2):
        exact = modes[:, m]
        got = Rz[1:-1, 0, m]
        assert np.abs(got - exact).max() < 1e-12 * np.abs(modes).max(), m
    assert np.abs(modes[:, 2]).max() > 1e-6       # the |grad z|^2 mode is really there


def test_variable_viscosity_mean_shear():
    """<m>1 = M(y), z = z0(y), rho D = 0, constant density: m^c = 0 and the
    RHS of <m>1 is (mu(z0) u1')' with u1 = M / rho0, at the interior points."""
    rho0 = 2.0
    mu_z = (4e-3, -2e-3, 1e-3)
    plan, w = make_plan(rho0, rho0, mu=1e-3, rhoD=0.0, mu_z=mu_z)
    h = plan.cfg.L2 / 2
    z0 = P([0.4, 0.08])
    M = P([0.0, 0.0, 0.0, -h * h / 6, 0.0, 1.0 / 60]) * 0.01
    st = zero_state(plan)
    st["z"][:, 0, 0] = interp(plan, z0)
    st["m1bar"] = interp(plan, M)
    out = run(plan, st)
    mu = 1e-3 + mu_z[0] * z0 + mu_z[1] * z0 ** 2 + mu_z[2] * z0 ** 3
    exact = (mu * (M / rho0).deriv()).deriv()
    tau = plan.sp.tau[1:-1]
    got = (plan.sp.E[0] @ out["rhs"]["m1bar"])[1:-1]
    assert np.abs(got - exact(tau)).max() < 1e-12 * np.abs(exact(tau)).max()


def test_variable_viscosity_single_mode_phi2_rhs():
    """m2^d one (l, n) mode (Robin quintic), Omega2 = 0, z = z0(y) linear,
    mu = mu0 + mu1 z, rho = f(z) of the mixture, so that 1/rho is linear in y
    and u = m/rho is a polynomial with theta = div u != 0.  k_f = 0 from a zero
    guess keeps m^c = 0.  The nonlinear terms miss (l, n), so RHS_phi2 there is
    the viscous part with T_ij = mu(y) S_ij."""
    rl, rh = 1.0, 3.0
    plan, w = make_plan(rl, rh, mu=2e-3, mu_z=(5e-3, 0.0, 0.0))
    ni, l = 12, 2
    k1 = float((plan.ik1 / 1j).real[0, 0, l])
    k3 = float((plan.ik3 / 1j).real[0, ni, 0])
    k2 = k1 * k1 + k3 * k3
    m2 = robin_poly(plan, ni, l, P([0.0, 0.0, 0.4, -0.1, 0.05, 0.01]))
    z0 = P([0.45, 0.05])
    rinv = (rh - (rh - rl) * z0) / (rl * rh)       # 1/rho along y
    amp = 0.5 - 0.2j
    st = zero_state(plan)
    st["z"][:, 0, 0] = interp(plan, z0)
    st["phi2"][:, ni, l] = amp * interp(plan, m2.deriv(2) - k2 * m2)
    out = run(plan, st, kf=0)
    assert all(np.abs(x).max() == 0 for x in out["diag"]["mc"])
    # divergence-free m^d of the mode with Omega2 = 0: m1 = i k1 m2'/k^2, m3 = i k3 m2'/k^2
    C = lambda p, c: P(np.asarray(p.coef, dtype=complex) * c)
    u = [C(m2.deriv(), amp * 1j * k1 / k2) * rinv, C(m2, amp) * rinv, C(m2.deriv(), amp * 1j * k3 / k2) * rinv]
    dx = [lambda p: C(p, 1j * k1), lambda p: p.deriv(), lambda p: C(p, 1j * k3)]
    d = [[dx[j](u[i]) for j in range(3)] for i in range(3)]      # d u_i / d x_j
    theta = d[0][0] + d[1][1] + d[2][2]
    mu = 2e-3 + 5e-3 * z0
    T = [[mu * (d[i][j] + d[j][i] - (2.0 / 3.0 * theta if i == j else 0)) for j in range(3)] for i in range(3)]
    N = [dx[0](T[i][0]) + T[i][1].deriv() + dx[2](T[i][2]) for i in range(3)]
    Rphi = C(N[1], -k2) - (dx[0](N[0]) + dx[2](N[2])).deriv()
    tau = plan.sp.tau[1:-1]
    got = apply(plan.sp.E[0], out["rhs"]["phi2"])[1:-1, ni, l]
    exact = Rphi(tau)
    assert np.abs(got - exact).max() < 1e-11 * np.abs(exact).max()
    assert np.abs(theta(tau)).max() > 1e-2 * np.abs(d[1][1](tau)).max()
    # and it is not the constant-mu result
    plan0, _ = make_plan(rl, rh, mu=2e-3)
    got0 = apply(plan0.sp.E[0], run(plan0, st, kf=0)["rhs"]["phi2"])[1:-1, ni, l]
    assert np.abs(got0 - exact).max() > 1e-2 * np.abs(exact).max()
