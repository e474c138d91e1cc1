"""Oracle of one explicit RK2 substep of the low-Mach variable-density method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path never
does, and it shares no code with the HIP library.

What it computes: one substep s -> s+1 of the time advance of the state
S = (phi2, Omega2, z, <m>1, <m>3) (Section 4 "Time advance", Algorithm
time_advanceDNS), written out step by step in the paper's order and notation,
in float64, with numpy/scipy library primitives (FFT, banded LU) as steps:

  1. finalize m^d: Poisson problem for m2^d (eq. phi_poisson) with the
     potential-matching Robin rows (eq. bc_both), then m1^d, m3^d from the
     divergence-free condition and Omega2 (eq. md_recon); the plane mean of m^d
     is (<m>1, 0, <m>3) (eq. mean_m1m3 and the sentence after it);
  2. R_z = -(1/rho) m^d . grad z + (1/rho) div(rho D grad z) (Section 2.1) and
     the BDF-like guess of dz/dt (eq. dzdt_guesses);
  3. k_f fixed-point iterations z_t^k = L(z) z_t^{k-1} + R_z (eq. y_k,
     Section 3.2), L applied matrix-free (Section 4.3): rho_t = f'(z) z_t, the
     curl-free momentum from the coupled mass / curl-free equations
     (eqs. COM_fourier, CF_fourier, mc_recon, mc_mean), then
     -(1/rho) grad z . m^c; then m^c from z_t^{k_f};
  4. rho = f(z) (equation of state of the Rayleigh-Taylor setup);
  5. RHS of Omega2, phi2 (eqs. om, phi, with the body force -rho g delta_i2)
     and of the plane means (eq. mean_m1m3);
  6. explicit midpoint RK2 in low-storage form.

Readings of points the paper leaves open (each is listed in the design notes):
  R1  RK2 = explicit midpoint: X' = X^n + dt/2 R^n, X^{n+1} = X' + dt (R' - R^n/2)
  R3  k_f applications of the fixed-point map, the guess being iterate 0
  R5  startup without history: zero guess and more iterations (a call option)
  R6  beta^n = 0, beta' = -4 (defaults)
  R7  3/2-rule physical grid, Nyquist modes excluded
  R9  collocation at Greville points: tau (B) for every field in B, tau* (B*)
      for the m2 equations
  R13 boundary rows replace the end collocation rows: Dirichlet for phi2,
      Omega2; Neumann for z_t, <m>1, <m>3; Robin for m2 (both parts)
  R14 <m2>(+L2/2) = 0
  R15 m^c: mass equation imposed exactly on the coefficients, curl-free
      equation collocated at the interior tau*
  R16 tau_ij from the projected u = m/rho.  The transport laws mu = g(z) and
      D_z = h(z) (Section 2) are cubic polynomials in z: g(z) = mu + sum_k
      mu_z[k] z^(k+1); rho D_z = q(z) or f(z) q(z) with q(z) = rhoD + sum_k
      rhoD_z[k] z^(k+1) (rhoD_form 0 / 1).  All zero: constant mu, rho D.
  R16b div(rho D grad z) is expanded by the chain rule, rho D lap z +
      (rho D)'(z) |grad z|^2, on the physical grid of the R_z product
  R17 RHS_phi2 = -k^2 N2 - d/dy(i k1 N1 + i k3 N3) + k^2 g rho
  R18 gravity uses rho = f(z) on the physical grid, forward-transformed
  R19 advective z equation as printed
  R25 rho^s = f(z^s) is formed before it is needed
  R26 m^c of the stage comes from one more rho_t -> m^c solve with z_t^{k_f}
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_banded

from .bspline import SplineSpaces
from .fourier import to_physical, to_spectral, wavenumbers


@dataclass
class Config:
    n1: int
    n3: int
    n2: int
    order: int
    m1: int
    m3: int
    L1: float
    L2: float
    L3: float
    breakpoints: np.ndarray
    dt: float
    mu: float
    rhoD: float
    g: float
    rho_l: float
    rho_h: float
    beta_n: float = 0.0
    beta_p: float = -4.0
    kf: int = 4
    mu_z: tuple = (0.0, 0.0, 0.0)
    rhoD_z: tuple = (0.0, 0.0, 0.0)
    rhoD_form: int = 0


# ----------------------------------------------------------------------------
# linear algebra helpers (library banded LU)


def _band_form(A: np.ndarray):
    """(lower, upper) bandwidths of A and its LAPACK band storage."""
    r, c = np.nonzero(A)
    lo = int(max(0, (r - c).max()))
    up = int(max(0, (c - r).max()))
    n = A.shape[0]
    ab = np.zeros((lo + up + 1, n))
    for i in range(n):
        for j in range(max(0, i - lo), min(n, i + up + 1)):
            ab[up + i - j, j] = A[i, j]
    return (lo, up), ab


def banded_solve(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve A X = B (A square, banded; B [n, ...] real or complex)."""
    lu, ab = _band_form(A)
    shp = B.shape
    X = solve_banded(lu, ab, B.reshape(shp[0], -1))
    return X.reshape(shp)


def apply(M: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Apply a y-matrix to the leading (y) axis of a field."""
    return np.tensordot(M, X, axes=(1, 0))


# ----------------------------------------------------------------------------


class Plan:
    """Constant tables of the discretisation (App. C; Section 4 eq. disc_f)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        if cfg.n1 % 2 or cfg.n3 % 2:
            raise ValueError("N1, N3 must be even")
        self.sp = SplineSpaces(cfg.breakpoints, cfg.order)
        if self.sp.n2 != cfg.n2:
            raise ValueError("breakpoint count does not match n2 and order")
        self.k1, self.k3, self.ksq = wavenumbers(cfg.n1, cfg.n3, cfg.L1, cfg.L3)
        self.k = np.sqrt(self.ksq)
        self.nn = cfg.n3 - 1
        self.nl = cfg.n1 // 2
        n2 = cfg.n2
        E = self.sp.E
        # projections values -> coefficients (R13)
        self.P_plain = E[0].copy()
        self.P_D = E[0].copy()
        self.P_D[0, :] = 0.0
        self.P_D[0, 0] = 1.0
        self.P_D[n2 - 1, :] = 0.0
        self.P_D[n2 - 1, n2 - 1] = 1.0
        self.P_N = E[0].copy()
        self.P_N[0, :] = E[1][0]
        self.P_N[n2 - 1, :] = E[1][n2 - 1]
        # multipliers of d/dx1, d/dx3 on [j, n_idx, l] arrays
        self.ik1 = (1j * self.k1)[None, None, :]
        self.ik3 = (1j * self.k3)[None, :, None]
        # mean-mode system of <m2^c>: D* c = -<rho_t>, c_top = 0 (R14)
        self.mean_m2 = np.vstack([self.sp.Dstar, np.eye(n2 + 1)[n2:n2 + 1]])

    # -- y operations ----------------------------------------------------------
    def A_of_k(self, k: float) -> np.ndarray:
        """(E*_2 - k^2 E*_0) with Robin rows k m2 -+ dm2/dy = 0 (eqs. phi_poisson, bc_both)."""
        Es = self.sp.Es
        n = self.cfg.n2 + 1
        A = Es[2] - k * k * Es[0]
        A[0, :] = k * Es[0][0] - Es[1][0]
        A[n - 1, :] = k * Es[0][n - 1] + Es[1][n - 1]
        return A

    def solve_A(self, R: np.ndarray) -> np.ndarray:
        """Solve A(k) c = R column by column for every (l, n) != (0, 0).

        Columns with the same k^2 share one banded LU.  The (0,0) column of the
        result is zero.
        """
        out = np.zeros_like(R)
        ksq = self.ksq.ravel()
        vals, inv = np.unique(ksq, return_inverse=True)
        order = np.argsort(inv, kind="stable")         # columns of each k^2 together, in row-major order
        bounds = np.searchsorted(inv[order], np.arange(len(vals) + 1))
        nl = self.ksq.shape[1]
        for g, val in enumerate(vals):
            if val == 0.0:
                continue
            flat = order[bounds[g]:bounds[g + 1]]
            idx = (flat // nl, flat % nl)
            A = self.A_of_k(np.sqrt(val))
            out[:, idx[0], idx[1]] = banded_solve(A, R[:, idx[0], idx[1]])
        return out

    def project(self, V: np.ndarray, kind: str) -> np.ndarray:
        """Values at tau -> B coefficients: 'plain' interpolation, or with the
        end rows replaced by homogeneous 'dirichlet' / 'neumann' conditions."""
        n2 = self.cfg.n2
        if kind == "plain":
            return banded_solve(self.P_plain, V)
        R = V.copy()
        R[0] = 0.0
        R[n2 - 1] = 0.0
        return banded_solve(self.P_D if kind == "dirichlet" else self.P_N, R)

    # -- physical-space phase --------------------------------------------------
    def plane_phase(self, inputs, func, batch_bytes=256 << 20):
        """Inverse-transform `inputs` (value arrays), apply the pointwise `func`
        to the physical fields and forward-transform its outputs.  Processed in
        batches of y-planes to bound memory; the arithmetic is per point."""
        c = self.cfg
        ny = inputs[0].shape[0]
        per_plane = 8 * c.m1 * c.m3 * (len(inputs) + 12)
        nb = max(1, min(ny, batch_bytes // per_plane))
        outs = None
        for j0 in range(0, ny, nb):
            j1 = min(ny, j0 + nb)
            phys = [to_physical(V[j0:j1], c.m1, c.m3) for V in inputs]
            res = func(*phys)
            spec = [to_spectral(r, c.n1, c.n3) for r in res]
            if outs is None:
                outs = [np.empty((ny,) + s.shape[1:], dtype=np.complex128) for s in spec]
            for o, s in zip(outs, spec):
                o[j0:j1] = s
        return outs

    # -- equation of state (Section 5, miscible RT mixing) ---------------------
    def rho_of_z(self, z):
        c = self.cfg
        return c.rho_l * c.rho_h / (c.rho_h - (c.rho_h - c.rho_l) * z)

    def drho_dz(self, rho):
        c = self.cfg
        return rho * rho * (c.rho_h - c.rho_l) / (c.rho_l * c.rho_h)

    # -- transport laws mu = g(z), rho D_z (Section 2; reading R16) -----------
    def mu_of_z(self, z):
        c = self.cfg
        return c.mu + c.mu_z[0] * z + c.mu_z[1] * z ** 2 + c.mu_z[2] * z ** 3

    def rhoD_of_z(self, z):
        """(rho D_z, d(rho D_z)/dz) at z."""
        c = self.cfg
        q = c.rhoD + c.rhoD_z[0] * z + c.rhoD_z[1] * z ** 2 + c.rhoD_z[2] * z ** 3
        dq = c.rhoD_z[0] + 2.0 * c.rhoD_z[1] * z + 3.0 * c.rhoD_z[2] * z ** 2
        if c.rhoD_form == 0:
            return q, dq
        rho = self.rho_of_z(z)
        return rho * q, self.drho_dz(rho) * q + rho * dq


# ----------------------------------------------------------------------------
# momentum decomposition


def divergence_free_momentum(plan: Plan, phi2, omega2, m1bar, m3bar):
    """m^d from (phi2, Omega2, <m>1, <m>3) (eqs. phi_poisson, md_recon, bc_both).

    Returns (m1 coefficients in B, m2 coefficients in B*, m3 coefficients in B).
    """
    sp = plan.sp
    n2 = plan.cfg.n2
    R = apply(sp.G[0], phi2)            # phi2 at tau*
    R[0] = 0.0
    R[n2] = 0.0                          # Robin rows
    c2 = plan.solve_A(R)
    dc2 = apply(sp.Dstar, c2)            # d m2 / dy in B (exact)
    ksq = np.where(plan.ksq == 0.0, 1.0, plan.ksq)[None]
    m1 = (plan.ik1 * dc2 - plan.ik3 * omega2) / ksq
    m3 = (plan.ik3 * dc2 + plan.ik1 * omega2) / ksq
    m1[:, 0, 0] = m1bar
    m3[:, 0, 0] = m3bar
    c2[:, 0, 0] = 0.0
    return m1, c2, m3


def curl_free_momentum(plan: Plan, rhot):
    """m^c from the B coefficients of rho_t (eqs. COM_fourier, CF_fourier,
    mc_recon, mc_mean; reading R15).

    Mass conservation rho_t + i k m_par + d m2/dy = 0 holds exactly on the
    coefficients; the curl-free equation d m_par/dy - i k m2 = 0 is collocated
    at the interior tau*, which gives (E*_2 - k^2 E*_0) c = -G_1 rho_t plus
    the Robin rows.  Returns (m1, m2 coefficients in B*, m3, m_par).
    """
    sp = plan.sp
    n2 = plan.cfg.n2
    R = -apply(sp.G[1], rhot)
    R[0] = 0.0
    R[n2] = 0.0
    c2 = plan.solve_A(R)
    k = np.where(plan.k == 0.0, 1.0, plan.k)[None]
    mpar = (1j / k) * (rhot + apply(sp.Dstar, c2))
    m1 = (plan.k1[None, None, :] / k) * mpar
    m3 = (plan.k3[None, :, None] / k) * mpar
    # plane mean: d<m2>/dy = -<rho_t>, <m2>(top) = 0, <m1> = <m3> = 0
    rhs = np.concatenate([-rhot[:, 0, 0], [0.0]])
    c2[:, 0, 0] = np.linalg.solve(plan.mean_m2, rhs)
    m1[:, 0, 0] = 0.0
    m3[:, 0, 0] = 0.0
    mpar[:, 0, 0] = 0.0
    return m1, c2, m3, mpar


# ----------------------------------------------------------------------------
# BDF-like initial guesses (eq. dzdt_guesses; Appendix A)


def bdf_coefficients(stage: int, beta_n: float = 0.0, beta_p: float = -4.0):
    """(a1, a2, a3, a4) with dt dz/dt^{s,0} = a1 z^s + a2 h1 + a3 h2 + a4 h3,
    h1, h2, h3 being the previous three stage values (most recent first)."""
    if stage == 0:
        return (2.0, -2.0 - 0.5 * beta_n, beta_n, -0.5 * beta_n)
    return (4.0 + beta_p, -5.0 - 2.0 * beta_p, beta_p, 1.0)


# ----------------------------------------------------------------------------
# the substep


def substep(plan: Plan, state: dict, stage: int, hist=None, rhs_prev=None,
            zt_prev=None, kf=None, guess="bdf", diagnostics=False):
    """One substep of Algorithm time_advanceDNS.

    state     dict: phi2, omega2, z  -> complex [n2, N3-1, N1/2] B coefficients;
              m1bar, m3bar -> real [n2] B coefficients of the plane means
    stage     0 (stage n: X' = X + dt/2 R) or 1 (stage ': X^{n+1} = X + dt (R - R^n/2))
    hist      (h1, h2, h3): z coefficients of the previous three stages
              (stage n: z^{n-1,'}, z^{n-1}, z^{n-2,'}; stage ': z^n, z^{n-1,'}, z^{n-1})
    rhs_prev  stage ' only: dict phi2, omega2, m1bar, m3bar of the stage-n RHS
    zt_prev   stage ' only: z_t^{n,k_f}
    kf        fixed-point iterations (default: the plan's)
    guess     'bdf' (eq. dzdt_guesses) or 'zero' (startup)

    Returns dict: state (new), rhs (this stage's RHS), zt (z_t^{s,k_f}) and,
    with diagnostics, the intermediate quantities.
    """
    c = plan.cfg
    sp = plan.sp
    E0, E1, E2 = sp.E
    F0 = sp.F[0]
    kf = c.kf if kf is None else kf
    ik1, ik3 = plan.ik1, plan.ik3
    ksq = plan.ksq[None]
    z = state["z"]
    diag = {}

    # 1. m^d
    md1, md2, md3 = divergence_free_momentum(plan, state["phi2"], state["omega2"],
                                             state["m1bar"], state["m3bar"])

    # values of z and its derivatives at tau
    Vz = apply(E0, z)
    Vz2 = apply(E1, z)
    Vlap = apply(E2, z) - ksq * Vz
    grad_z = [ik1 * Vz, Vz2, ik3 * Vz]

    # 2. R_z
    def rz(zp, z1, z2, z3, lap, m1, m2, m3):
        rho = plan.rho_of_z(zp)
        k, dk = plan.rhoD_of_z(zp)
        diff = k * lap + dk * (z1 * z1 + z2 * z2 + z3 * z3)      # div(rho D grad z), R16b
        return [(-(m1 * z1 + m2 * z2 + m3 * z3) + diff) / rho]

    (VR,) = plan.plane_phase([Vz] + grad_z + [Vlap, apply(E0, md1), apply(F0, md2),
                                              apply(E0, md3)], rz)
    Rz = plan.project(VR, "neumann")

    # BDF-like guess (or zero at startup)
    if guess == "bdf":
        a = bdf_coefficients(stage, c.beta_n, c.beta_p)
        zt = (a[0] * z + a[1] * hist[0] + a[2] * hist[1] + a[3] * hist[2]) / c.dt
    else:
        zt = np.zeros_like(z)
    if diagnostics:
        diag["Rz"] = Rz
        diag["zt0"] = zt.copy()
        diag["increments"] = []

    def rho_t_of(zt_coef):
        def prod(zp, ztp):
            return [plan.drho_dz(plan.rho_of_z(zp)) * ztp]
        (Vrt,) = plan.plane_phase([Vz, apply(E0, zt_coef)], prod)
        return plan.project(Vrt, "plain")

    def L_apply(mc1, mc2, mc3):
        def prod(zp, z1, z2, z3, m1, m2, m3):
            rho = plan.rho_of_z(zp)
            return [-(z1 * m1 + z2 * m2 + z3 * m3) / rho]
        (VL,) = plan.plane_phase([Vz] + grad_z + [apply(E0, mc1), apply(F0, mc2),
                                                  apply(E0, mc3)], prod)
        return plan.project(VL, "neumann")

    # 3. fixed-point iterations z_t^k = L(z) z_t^{k-1} + R_z
    for _ in range(kf):
        rhot = rho_t_of(zt)
        mc1, mc2, mc3, _ = curl_free_momentum(plan, rhot)
        zt_new = L_apply(mc1, mc2, mc3) + Rz
        if diagnostics:
            diag["increments"].append(float(np.abs(zt_new - zt).max()))
        zt = zt_new
    rhot = rho_t_of(zt)
    mc1, mc2, mc3, mpar = curl_free_momentum(plan, rhot)
    if diagnostics:
        diag.update(md=(md1, md2, md3), mc=(mc1, mc2, mc3), rhot=rhot, mpar=mpar)

    # 4./5. momentum fluxes and right-hand sides
    m1 = md1 + mc1
    m2 = md2 + mc2
    m3 = md3 + mc3
    Vm = [apply(E0, m1), apply(F0, m2), apply(E0, m3)]

    def velocities(zp, p1, p2, p3):
        rho = plan.rho_of_z(zp)
        return [p1 / rho, p2 / rho, p3 / rho, rho]

    Vu1, Vu2, Vu3, Vrho = plan.plane_phase([Vz] + Vm, velocities)
    u = [plan.project(V, "plain") for V in (Vu1, Vu2, Vu3)]
    du = []                                   # du[i][j] = d u_i / d x_j
    for ui in u:
        V0 = apply(E0, ui)
        du.append([ik1 * V0, apply(E1, ui), ik3 * V0])
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]

    def fluxes(zp, p1, p2, p3, *g):
        rho = plan.rho_of_z(zp)
        mu = plan.mu_of_z(zp)
        m = (p1, p2, p3)
        d = [g[0:3], g[3:6], g[6:9]]
        theta = d[0][0] + d[1][1] + d[2][2]
        out = []
        for i, j in pairs:
            t = -m[i] * m[j] / rho + mu * (d[i][j] + d[j][i])
            if i == j:
                t = t - (2.0 / 3.0) * mu * theta
            out.append(t)
        return out

    VT = plan.plane_phase([Vz] + Vm + [x for row in du for x in row], fluxes)
    Th = [plan.project(V, "plain") for V in VT]
    T = {}
    for (i, j), t in zip(pairs, Th):
        T[(i, j)] = t
        T[(j, i)] = t

    # N_i = d_j T_ij and its y-derivative, as values at tau
    Nv, dNv = [], []
    for i in range(3):
        Nv.append(ik1 * apply(E0, T[(i, 0)]) + apply(E1, T[(i, 1)]) + ik3 * apply(E0, T[(i, 2)]))
        dNv.append(ik1 * apply(E1, T[(i, 0)]) + apply(E2, T[(i, 1)]) + ik3 * apply(E1, T[(i, 2)]))
    R_omega = ik3 * Nv[0] - ik1 * Nv[2]                          # eq. om
    R_phi = -ksq * Nv[1] - (ik1 * dNv[0] + ik3 * dNv[2]) + ksq * c.g * Vrho   # eq. phi (R17)
    R_omega[:, 0, 0] = 0.0
    R_phi[:, 0, 0] = 0.0
    rhs = {
        "phi2": plan.project(R_phi, "dirichlet"),
        "omega2": plan.project(R_omega, "dirichlet"),
        "m1bar": plan.project(apply(E1, T[(0, 1)][:, 0, 0].real), "neumann"),
        "m3bar": plan.project(apply(E1, T[(2, 1)][:, 0, 0].real), "neumann"),
    }
    rhs["phi2"][:, 0, 0] = 0.0
    rhs["omega2"][:, 0, 0] = 0.0
    if diagnostics:
        diag.update(u=u, T=Th, rho_vals=Vrho)

    # 6. RK2 (explicit midpoint, low-storage form)
    new = {}
    keys = ("phi2", "omega2", "m1bar", "m3bar")
    if stage == 0:
        for key in keys:
            new[key] = state[key] + 0.5 * c.dt * rhs[key]
        new["z"] = z + 0.5 * c.dt * zt
    else:
        for key in keys:
            new[key] = state[key] + c.dt * (rhs[key] - 0.5 * rhs_prev[key])
        new["z"] = z + c.dt * (zt - 0.5 * zt_prev)
    out = {"state": new, "rhs": rhs, "zt": zt}
    if diagnostics:
        out["diag"] = diag
    return out


class Integrator:
    """Drives substeps with the z history and stored stage data (eq. before
    Algorithm time_advanceDNS).  Step 0 has no history and uses the startup
    path (zero guess, `k_startup` iterations) for both of its stages."""

    def __init__(self, plan: Plan, state: dict, k_startup: int = 40, hist=None):
        self.plan = plan
        self.state = {k: v.copy() for k, v in state.items()}
        self.k_startup = k_startup
        self.hist = list(hist) if hist is not None else None  # [h1, h2, h3]
        self.step_count = 0

    def step(self):
        p = self.plan
        startup = self.hist is None
        z_n = self.state["z"].copy()
        kw = dict(kf=self.k_startup, guess="zero") if startup else dict(hist=self.hist)
        a = substep(p, self.state, 0, **kw)
        hist_p = [z_n] + (self.hist[:2] if self.hist else [z_n, z_n])
        z_p = a["state"]["z"].copy()
        kw = dict(kf=self.k_startup, guess="zero") if startup else dict(hist=hist_p)
        b = substep(p, a["state"], 1, rhs_prev=a["rhs"], zt_prev=a["zt"], **kw)
        self.hist = [z_p, z_n, hist_p[1]]
        self.state = b["state"]
        self.step_count += 1
        return self.state
