"""Oracle of the adjoint (reverse mode) of one substep.

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module; the
product path never does, and it shares no code with the HIP library.

The substep (Algorithm time_advanceDNS, as computed by oracle.lmvd.substep) is
a composition of linear operators (evaluation E_d and F_0, the inverse and
forward transforms on the 3/2 grid, the projections, m^d and m^c, spectral
multipliers) and pointwise products on the grid (R_z and L z_t of Sections 2.1
and 4.3, rho_t = f'(z) z_t, u = m/rho, C_ij = -m_i m_j/rho).  Its adjoint is the
composition of the transposes in reverse order.  Transposes are taken in the
real inner products <a, b> = sum Re(conj(a) b) over the stored entries of a
spectral array and the plain sum over a physical field or a real vector.

Each transpose below is written from the definition of its operator:
  E_d, F_0, projections      matrix transposes (P^{-T}, then the end rows zeroed)
  inverse transform          u = sum_{stored (l,n)} w_l Re(V e^{i(k1 x + k3 z)}),
                             w_0 = 1, w_l = 2: transpose V_bar = w_l M1 M3 Fwd(u_bar)
  forward transform          V = Fwd(u): transpose u_bar = Inv(V_bar / w_l) / (M1 M3)
  complex multiplier c       transpose conj(c)
  m^d, m^c                   the A(k) solve transposed (A(k)^{-T}), D*^T, G_0^T, G_1^T,
                             the conjugated multipliers; the plane-mean systems
                             transposed
  pointwise products         their Jacobians (derivatives of the products in z,
                             grad z, lap z, m, z_t on the grid)
Only constant transport coefficients (mu, rho D) are covered.
"""
from __future__ import annotations

import numpy as np

from .fourier import to_physical, to_spectral
from .lmvd import apply, bdf_coefficients, curl_free_momentum, divergence_free_momentum


# ----------------------------------------------------------------------------
# transposes of the linear operators


def weights(plan):
    """w_l of the inverse transform: 1 for l = 0, 2 for l > 0."""
    w = np.full(plan.nl, 2.0)
    w[0] = 1.0
    return w[None, None, :]


def to_physical_t(plan, ub):
    """Transpose of the inverse transform: physical cotangent -> values cotangent."""
    c = plan.cfg
    return weights(plan) * (c.m1 * c.m3) * to_spectral(ub, c.n1, c.n3)


def to_spectral_t(plan, Vb):
    """Transpose of the forward transform: values cotangent -> physical cotangent."""
    c = plan.cfg
    return to_physical(Vb / weights(plan), c.m1, c.m3) / (c.m1 * c.m3)


def apply_t(M, Xb):
    """Transpose of applying the real y-matrix M."""
    return np.tensordot(M.T, Xb, axes=(1, 0))


def project_t(plan, Xb, kind):
    """Transpose of plan.project(V, kind): R P^{-T} with R the end-row replacement."""
    P = {"plain": plan.P_plain, "dirichlet": plan.P_D, "neumann": plan.P_N}[kind]
    shp = Xb.shape
    V = np.linalg.solve(P.T, Xb.reshape(shp[0], -1)).reshape(shp)
    if kind != "plain":
        V[0] = 0.0
        V[-1] = 0.0
    return V


def solve_A_t(plan, Cb):
    """Transpose of plan.solve_A: A(k)^{-T} per column, (0,0) column zero."""
    out = np.zeros_like(Cb)
    for val in np.unique(plan.ksq):
        if val == 0.0:
            continue
        idx = np.nonzero(plan.ksq == val)
        A = plan.A_of_k(np.sqrt(val))
        out[:, idx[0], idx[1]] = np.linalg.solve(A.T, Cb[:, idx[0], idx[1]])
    return out


def md_t(plan, m1b, c2b, m3b):
    """Transpose of divergence_free_momentum: (m1, m2 in B*, m3) cotangents -> (phi2, Omega2, <m>1, <m>3)."""
    sp = plan.sp
    n2 = plan.cfg.n2
    ksq = np.where(plan.ksq == 0.0, 1.0, plan.ksq)[None]
    # m1 = (i k1 D - i k3 Om) / k^2, m3 = (i k3 D + i k1 Om) / k^2
    Db = (np.conj(plan.ik1) * m1b + np.conj(plan.ik3) * m3b) / ksq
    Omb = (np.conj(-plan.ik3) * m1b + np.conj(plan.ik1) * m3b) / ksq
    Db[:, 0, 0] = 0.0
    Omb[:, 0, 0] = 0.0
    cb = c2b.copy()
    cb[:, 0, 0] = 0.0
    cb = cb + apply_t(sp.Dstar, Db)
    Rb = solve_A_t(plan, cb)
    Rb[0] = 0.0
    Rb[n2] = 0.0
    phib = apply_t(sp.G[0], Rb)
    phib[:, 0, 0] = 0.0
    return phib, Omb, m1b[:, 0, 0].real.copy(), m3b[:, 0, 0].real.copy()


def mc_t(plan, m1b, c2b, m3b):
    """Transpose of curl_free_momentum (its first three outputs): -> rho_t cotangent."""
    sp = plan.sp
    n2 = plan.cfg.n2
    k = np.where(plan.k == 0.0, 1.0, plan.k)[None]
    mparb = (plan.k1[None, None, :] / k) * m1b + (plan.k3[None, :, None] / k) * m3b
    mparb[:, 0, 0] = 0.0
    Sb = np.conj(1j / k) * mparb                  # cotangent of rho_t + D* c
    cb = c2b.copy()
    cb[:, 0, 0] = 0.0
    cb = cb + apply_t(sp.Dstar, Sb)
    Rb = solve_A_t(plan, cb)
    Rb[0] = 0.0
    Rb[n2] = 0.0
    rhotb = Sb - apply_t(sp.G[1], Rb)
    # plane mean: c2 = M^{-1} [-rho_t; 0]
    mb = np.linalg.solve(plan.mean_m2.T, c2b[:, 0, 0])
    rhotb[:, 0, 0] = -mb[:n2]
    return rhotb


def hermitian(a, zero00=False):
    """The representative with a Hermitian l = 0 column: (a_{0,n} + conj a_{0,-n}) / 2; (0,0) real (or 0)."""
    a = a.copy()
    nn = a.shape[1]
    for ni in range(1, (nn + 1) // 2):
        h = 0.5 * (a[:, ni, 0] + np.conj(a[:, nn - ni, 0]))
        a[:, ni, 0] = h
        a[:, nn - ni, 0] = np.conj(h)
    a[:, 0, 0] = 0.0 if zero00 else a[:, 0, 0].real
    return a


# ----------------------------------------------------------------------------
# the substep's adjoint


def substep_adjoint(plan, state, stage, cot, hist=None, rhs_prev=None, zt_prev=None, kf=None, guess="bdf"):
    """Gradients of <cot, substep outputs> with respect to the substep's inputs.

    state, stage, hist, rhs_prev, zt_prev, kf, guess: as for oracle.lmvd.substep.
    cot: dict of output cotangents: state (phi2, omega2, z, m1bar, m3bar), rhs (phi2, omega2, m1bar,
    m3bar), zt, and optionally md, mc (3-tuples, m2 in B*).
    Returns dict: phi2, omega2, z, m1bar, m3bar, hist (3, or None), and at stage 1 rhs_prev (dict),
    zt_prev.  S-field gradients are the representatives with a Hermitian l = 0 column; the (0,0)
    entries of the phi2, Omega2 gradients are zero."""
    c = plan.cfg
    sp = plan.sp
    E0, E1, E2 = sp.E
    F0 = sp.F[0]
    kf = c.kf if kf is None else kf
    ik1, ik3 = plan.ik1, plan.ik3
    ksq = plan.ksq[None]
    m1g, m3g = c.m1, c.m3
    inv = lambda V: to_physical(V, m1g, m3g)
    fwd = lambda u: to_spectral(u, c.n1, c.n3)
    inv_t = lambda u: to_physical_t(plan, u)
    fwd_t = lambda V: to_spectral_t(plan, V)
    z = state["z"]
    dr = c.rho_h - c.rho_l

    def rinv_of(zp):                      # 1 / rho = (rho_h - (rho_h - rho_l) z) / (rho_l rho_h)
        return (c.rho_h - dr * zp) / (c.rho_l * c.rho_h)

    def fprime(zp):                       # f'(z) = rho^2 (rho_h - rho_l) / (rho_l rho_h)
        r = 1.0 / rinv_of(zp)
        return r * r * dr / (c.rho_l * c.rho_h)

    # ---- forward, keeping what the transposes need ----
    md1, md2, md3 = divergence_free_momentum(plan, state["phi2"], state["omega2"], state["m1bar"], state["m3bar"])
    Vz = apply(E0, z)
    zp = inv(Vz)
    g = [inv(ik1 * Vz), inv(apply(E1, z)), inv(ik3 * Vz)]
    lap = inv(apply(E2, z) - ksq * Vz)
    mdp = [inv(apply(E0, md1)), inv(apply(F0, md2)), inv(apply(E0, md3))]
    rinv = rinv_of(zp)
    R = (-(mdp[0] * g[0] + mdp[1] * g[1] + mdp[2] * g[2]) + c.rhoD * lap) * rinv
    Rz = plan.project(fwd(R), "neumann")
    if guess == "bdf":
        a = bdf_coefficients(stage, c.beta_n, c.beta_p)
        zt = (a[0] * z + a[1] * hist[0] + a[2] * hist[1] + a[3] * hist[2]) / c.dt
    else:
        a = None
        zt = np.zeros_like(z)
    fp = fprime(zp)
    ztp, mcp = [], []
    for _ in range(kf):
        ztp.append(inv(apply(E0, zt)))
        rhot = plan.project(fwd(fp * ztp[-1]), "plain")
        mc = curl_free_momentum(plan, rhot)[:3]
        mcp.append([inv(apply(E0, mc[0])), inv(apply(F0, mc[1])), inv(apply(E0, mc[2]))])
        L = -(g[0] * mcp[-1][0] + g[1] * mcp[-1][1] + g[2] * mcp[-1][2]) * rinv
        zt = plan.project(fwd(L), "neumann") + Rz
    ztp.append(inv(apply(E0, zt)))
    rhot = plan.project(fwd(fp * ztp[-1]), "plain")
    mc = curl_free_momentum(plan, rhot)[:3]
    m = [md1 + mc[0], md2 + mc[1], md3 + mc[2]]
    mp = [inv(apply(E0, m[0])), inv(apply(F0, m[1])), inv(apply(E0, m[2]))]

    # ---- reverse ----
    cs, cr = cot["state"], cot["rhs"]
    w_out = 0.5 * c.dt if stage == 0 else c.dt
    Rphib = hermitian(cr["phi2"] + w_out * cs["phi2"], True)
    Romb = hermitian(cr["omega2"] + w_out * cs["omega2"], True)
    Rm1b = cr["m1bar"] + w_out * cs["m1bar"]
    Rm3b = cr["m3bar"] + w_out * cs["m3bar"]
    ztb = hermitian(cot["zt"] + w_out * cs["z"])
    zb = cs["z"].copy()
    out = {}
    if stage == 1:
        out["rhs_prev"] = {"phi2": hermitian(-0.5 * c.dt * cs["phi2"], True),
                           "omega2": hermitian(-0.5 * c.dt * cs["omega2"], True),
                           "m1bar": -0.5 * c.dt * cs["m1bar"], "m3bar": -0.5 * c.dt * cs["m3bar"]}
        out["zt_prev"] = hermitian(-0.5 * c.dt * cs["z"])

    # right-hand sides
    mask = np.ones(Vz.shape[1:])
    mask[0, 0] = 0.0
    vphi = mask * project_t(plan, Rphib, "dirichlet")
    vom = mask * project_t(plan, Romb, "dirichlet")
    Nb = [np.conj(ik3) * vom, np.conj(-ksq) * vphi, np.conj(-ik1) * vom]
    dNb = [np.conj(-ik1) * vphi, None, np.conj(-ik3) * vphi]
    rhob_vals = ksq * c.g * vphi
    pairs = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    pid = lambda i, j: pairs[(min(i, j), max(i, j))]
    Tb = [np.zeros_like(Vz) for _ in range(6)]
    for i in range(3):
        Tb[pid(i, 0)] += apply_t(E0, np.conj(ik1) * Nb[i])
        Tb[pid(i, 1)] += apply_t(E1, Nb[i])
        Tb[pid(i, 2)] += apply_t(E0, np.conj(ik3) * Nb[i])
        if dNb[i] is not None:
            Tb[pid(i, 0)] += apply_t(E1, np.conj(ik1) * dNb[i])
            Tb[pid(i, 1)] += apply_t(E2, dNb[i])
            Tb[pid(i, 2)] += apply_t(E1, np.conj(ik3) * dNb[i])
    for q, Rb in ((1, Rm1b), (4, Rm3b)):
        v = project_t(plan, Rb[:, None, None].astype(complex), "neumann")[:, 0, 0].real
        Tb[q][:, 0, 0] += apply_t(E1, v)
    # T_hat = P0^{-1} Fwd(T), T = -m_i m_j / rho + mu (d_ij + d_ji) - 2/3 mu theta delta_ij
    Vb = [project_t(plan, t, "plain") for t in Tb]
    Tgb = [fwd_t(v) for v in Vb]
    # viscous part: d_ij = Inv(D_j u_hat_i) = d u_i / d x_j, D = (i k1 E0, E1, i k3 E0)
    Dt = [lambda v: apply_t(E0, np.conj(ik1) * v), lambda v: apply_t(E1, v),
          lambda v: apply_t(E0, np.conj(ik3) * v)]
    db = [[np.zeros_like(zp) for _ in range(3)] for _ in range(3)]
    thetab = np.zeros_like(zp)
    for (i, j), q in pairs.items():
        if i == j:
            db[i][i] += 2.0 * c.mu * Tgb[q]
            thetab += -(2.0 / 3.0) * c.mu * Tgb[q]
        else:
            db[i][j] += c.mu * Tgb[q]
            db[j][i] += c.mu * Tgb[q]
    for i in range(3):
        db[i][i] += thetab
    uhb = [sum(Dt[j](inv_t(db[i][j])) for j in range(3)) for i in range(3)]
    # u_hat = P0^{-1} Fwd(m / rho)
    ub = [fwd_t(project_t(plan, x, "plain")) for x in uhb]
    # convective part T_ij = -m_i m_j / rho over the stored pairs, and u = m / rho
    mpb = [ub[i] * rinv for i in range(3)]
    rhob = fwd_t(rhob_vals)
    for (i, j), q in pairs.items():
        if i == j:
            mpb[i] = mpb[i] - 2.0 * Tgb[q] * mp[i] * rinv
        else:
            mpb[i] = mpb[i] - Tgb[q] * mp[j] * rinv
            mpb[j] = mpb[j] - Tgb[q] * mp[i] * rinv
        rhob = rhob + Tgb[q] * mp[i] * mp[j] * rinv * rinv
    rhob = rhob - rinv * rinv * (ub[0] * mp[0] + ub[1] * mp[1] + ub[2] * mp[2])
    zpb = rhob * fp
    mb = [apply_t(E0, inv_t(mpb[0])), apply_t(F0, inv_t(mpb[1])), apply_t(E0, inv_t(mpb[2]))]
    mdb = [x.copy() for x in mb]
    mcb = [x.copy() for x in mb]
    if cot.get("md") is not None:
        mdb = [x + y for x, y in zip(mdb, cot["md"])]
    if cot.get("mc") is not None:
        mcb = [x + y for x, y in zip(mcb, cot["mc"])]

    gb = [np.zeros_like(zp) for _ in range(3)]

    def rhot_t(k, mcb_):
        nonlocal zpb
        rb = fwd_t(project_t(plan, mc_t(plan, *mcb_), "plain"))
        fpp = 2.0 * fp * dr * (1.0 / rinv) / (c.rho_l * c.rho_h)
        zpb = zpb + fpp * ztp[k] * rb
        return apply_t(E0, inv_t(fp * rb))

    ztb = ztb + rhot_t(kf, mcb)
    Rzb = np.zeros_like(Vz)
    for k in range(kf - 1, -1, -1):
        Rzb = Rzb + ztb
        Lb = fwd_t(project_t(plan, ztb, "neumann"))
        a_sum = g[0] * mcp[k][0] + g[1] * mcp[k][1] + g[2] * mcp[k][2]
        mcpb = [-Lb * rinv * g[i] for i in range(3)]
        for i in range(3):
            gb[i] = gb[i] - Lb * rinv * mcp[k][i]
        zpb = zpb - Lb * (-dr / (c.rho_l * c.rho_h)) * a_sum
        mcb_k = [apply_t(E0, inv_t(mcpb[0])), apply_t(F0, inv_t(mcpb[1])), apply_t(E0, inv_t(mcpb[2]))]
        ztb = rhot_t(k, mcb_k)
    if guess == "bdf":
        zb = zb + (a[0] / c.dt) * ztb
        out["hist"] = [hermitian((a[h + 1] / c.dt) * ztb) for h in range(3)]
    else:
        out["hist"] = None
    # R_z
    Rb = fwd_t(project_t(plan, Rzb, "neumann"))
    a_R = -(mdp[0] * g[0] + mdp[1] * g[1] + mdp[2] * g[2]) + c.rhoD * lap
    mdpb = [-Rb * rinv * g[i] for i in range(3)]
    for i in range(3):
        gb[i] = gb[i] - Rb * rinv * mdp[i]
    lapb = Rb * rinv * c.rhoD
    zpb = zpb + Rb * (-dr / (c.rho_l * c.rho_h)) * a_R
    mdb[0] = mdb[0] + apply_t(E0, inv_t(mdpb[0]))
    mdb[1] = mdb[1] + apply_t(F0, inv_t(mdpb[1]))
    mdb[2] = mdb[2] + apply_t(E0, inv_t(mdpb[2]))
    # z on the grid
    zb = zb + apply_t(E0, inv_t(zpb) + np.conj(ik1) * inv_t(gb[0]) + np.conj(ik3) * inv_t(gb[2])
                      - ksq * inv_t(lapb))
    zb = zb + apply_t(E1, inv_t(gb[1])) + apply_t(E2, inv_t(lapb))
    phib, omb, m1b, m3b = md_t(plan, *mdb)
    out["phi2"] = hermitian(phib + cs["phi2"], True)
    out["omega2"] = hermitian(omb + cs["omega2"], True)
    out["m1bar"] = m1b + cs["m1bar"]
    out["m3bar"] = m3b + cs["m3bar"]
    out["z"] = hermitian(zb)
    return out
