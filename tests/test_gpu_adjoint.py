"""Adjoints of the linear operators (lmvd_to_physical_adjoint,
lmvd_to_spectral_adjoint, lmvd_evaluate_adjoint, lmvd_project_adjoint,
lmvd_md_adjoint, lmvd_mc_adjoint) and automatic differentiation through them
(paper_2206_09878_amd.autograd), through the C ABI:

  * <A x, y> = <x, A^T y> in the real inner products for the inverse transform
    (register and generic kernels), E_0, E_1, E_2, F_0 and the three
    projections, on random S-fields with a Hermitian l = 0 column (the inputs
    the library accepts);
  * E_d^T and the projections' transposes equal the oracle's dense transposes
    column by column (1e-12);
  * the gradient of a real loss through project -> evaluate -> to_physical
    matches central finite differences (eps = 1e-6) on 16 random directions;
  * m^d and m^c transposes against dot products and the oracle's dense maps;
  * one fixed-point iteration composed from the differentiable operators has
    the gradient of central differences.
"""
import numpy as np
import pytest

from oracle.lmvd import Plan as OPlan
from paper_2206_09878_amd.workloads import workload
from tests.conftest import oracle_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def rdot(torch, a, b):
    return float(torch.sum(torch.view_as_real(a) * torch.view_as_real(b)).item()) if a.is_complex() \
        else float(torch.sum(a * b).item())


def crand(torch, shape, seed):
    """Random S-field whose l = 0 column is Hermitian (f(0, -n) = conj f(0, n)), as the library's
    inputs must be."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    re = torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
    im = torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
    c = torch.complex(re, im)
    nn = shape[1]
    c[:, 0, 0] = c[:, 0, 0].real.to(c.dtype)
    for n in range(1, (nn + 1) // 2 + 1):
        if nn - n > n - 1:
            c[:, nn - n, 0] = torch.conj(c[:, n, 0])
    return c


def plan_of(n, n2):
    from paper_2206_09878_amd.lmvd import Plan
    return Plan(workload("small", n=n, n2=n2))


@pytest.mark.parametrize("n,n2", [(32, 33), (24, 25)])     # register and generic transform kernels
def test_transform_transpose(torch, n, n2):
    p = plan_of(n, n2)
    w = p.w
    c = crand(torch, w.shape, 1)
    g = torch.randn((w.n2, w.m3, w.m1), dtype=torch.float64, device="cuda")
    lhs = rdot(torch, p.to_physical(c), g)
    rhs = rdot(torch, c, p.to_physical_adjoint(g))
    torch.cuda.synchronize()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12
    # the forward transform's transpose
    lhs = rdot(torch, p.to_spectral(g), c)
    rhs = rdot(torch, g, p.to_spectral_adjoint(c))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12


@pytest.mark.parametrize("deriv,star", [(0, False), (1, False), (2, False), (0, True)])
def test_evaluate_transpose(torch, deriv, star):
    p = plan_of(32, 33)
    w = p.w
    c = crand(torch, w.shape_star if star else w.shape, 2)
    v = crand(torch, w.shape, 3)
    lhs = rdot(torch, p.evaluate(deriv, c, star=star), v)
    ct = p.evaluate_adjoint(deriv, v, star=star)
    rhs = rdot(torch, c, ct)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    # against the oracle's dense matrix, column by column
    op = OPlan(oracle_config(w))
    M = op.sp.F[0] if star else op.sp.E[deriv]
    ref = np.tensordot(M.T, v.cpu().numpy(), axes=(1, 0))
    got = ct.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,n2", [(32, 33), (16, 14), (16, 15), (16, 16), (16, 19)])  # row counts mod 4
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_project_transpose(torch, kind, n, n2):
    p = plan_of(n, n2)
    w = p.w
    v = crand(torch, w.shape, 4)
    y = crand(torch, w.shape, 5)
    lhs = rdot(torch, p.project(kind, v), y)
    vt = p.project_adjoint(kind, y)
    rhs = rdot(torch, v, vt)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    op = OPlan(oracle_config(w))
    A = (op.P_plain, op.P_D, op.P_N)[kind]
    yy = y.cpu().numpy()
    ref = np.linalg.solve(A.T, yy.reshape(w.n2, -1)).reshape(yy.shape)
    if kind:
        ref[0] = 0.0
        ref[-1] = 0.0
    got = vt.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_gradient_matches_central_differences(torch):
    """Loss = sum(W * to_physical(E_1 P_N v)): its gradient by autograd (the
    adjoint chain) against (L(v + eps d) - L(v - eps d)) / (2 eps) on 16 random
    directions d, eps = 1e-6."""
    from paper_2206_09878_amd.autograd import evaluate, project, to_physical
    p = plan_of(32, 33)
    w = p.w
    Wt = torch.randn((w.n2, w.m3, w.m1), dtype=torch.float64, device="cuda")

    def loss(v):
        return torch.sum(Wt * to_physical(p, evaluate(p, 1, project(p, 2, v))))

    v = crand(torch, w.shape, 6).requires_grad_(True)
    L = loss(v)
    L.backward()
    grad = v.grad.detach()
    eps = 1e-6
    with torch.no_grad():
        for k in range(16):
            d = crand(torch, w.shape, 100 + k)
            fd = (loss(v + eps * d) - loss(v - eps * d)).item() / (2 * eps)
            an = rdot(torch, grad, d)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (k, fd, an)


@pytest.mark.parametrize("n,n2", [(32, 33), (48, 49), (16, 14), (16, 19)])
def test_md_transpose(torch, n, n2):
    """<md(x), y> = <x, md^T(y)> for x = (phi2, Omega2, <m>1, <m>3) and y = (m1, m2 in B*, m3); and
    md^T against the oracle's m^d written as a dense real matrix on one column."""
    p = plan_of(n, n2)
    w = p.w
    phi, om = crand(torch, w.shape, 7), crand(torch, w.shape, 8)
    b1 = torch.randn(w.n2, dtype=torch.float64, device="cuda")
    b3 = torch.randn(w.n2, dtype=torch.float64, device="cuda")
    y1, y2, y3 = crand(torch, w.shape, 9), crand(torch, w.shape_star, 10), crand(torch, w.shape, 11)
    m1, m2, m3 = p.md(phi, om, b1, b3)
    lhs = rdot(torch, m1, y1) + rdot(torch, m2, y2) + rdot(torch, m3, y3)
    tp, to, t1, t3 = p.md_adjoint(y1, y2, y3)
    rhs = rdot(torch, phi, tp) + rdot(torch, om, to) + rdot(torch, b1, t1) + rdot(torch, b3, t3)
    torch.cuda.synchronize()
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs)), (lhs, rhs)
    # one column (l, n) = (3, 2) through the oracle, as a dense matrix of phi2 -> m2 (real and imaginary
    # unit inputs): its transpose applied to y2's column equals phi2_bar's column (from the m2 part)
    from oracle.lmvd import divergence_free_momentum
    op = OPlan(oracle_config(w))
    ni, l = 2, 3
    z = np.zeros(w.shape, dtype=complex)
    zb = np.zeros(w.n2)
    y2c = y2.cpu().numpy()[:, ni, l]
    cols = []
    for k in range(2 * w.n2):
        e = np.zeros(w.shape, dtype=complex)
        e[k % w.n2, ni, l] = 1.0 if k < w.n2 else 1j
        cols.append(divergence_free_momentum(op, e, z, zb, zb)[1][:, ni, l])
    A = np.array(cols).T                                   # m2 column (complex) <- (Re, Im) of phi2 column
    Ar = np.vstack([A.real, A.imag])                       # real form
    g = Ar.T @ np.concatenate([y2c.real, y2c.imag])
    zero = torch.zeros_like(y1)
    tp2 = p.md_adjoint(zero, y2, zero)[0].cpu().numpy()[:, ni, l]
    assert np.abs(tp2 - (g[:w.n2] + 1j * g[w.n2:])).max() < 1e-10 * np.abs(g).max()


@pytest.mark.parametrize("n,n2", [(32, 33), (48, 49), (16, 14), (16, 19)])
def test_mc_transpose(torch, n, n2):
    """<mc(rho_t), y> = <rho_t, mc^T(y)> (the (0,0) column with its plane-mean system included), and
    mc^T against the oracle's m^c written as a dense real matrix on one column and on the mean column."""
    p = plan_of(n, n2)
    w = p.w
    r = crand(torch, w.shape, 12)
    y1, y2, y3 = crand(torch, w.shape, 13), crand(torch, w.shape_star, 14), crand(torch, w.shape, 15)
    m1, m2, m3 = p.mc(r)
    lhs = rdot(torch, m1, y1) + rdot(torch, m2, y2) + rdot(torch, m3, y3)
    rt = p.mc_adjoint(y1, y2, y3)
    rhs = rdot(torch, r, rt)
    torch.cuda.synchronize()
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs)), (lhs, rhs)
    from oracle.lmvd import curl_free_momentum
    op = OPlan(oracle_config(w))
    ys = [y.cpu().numpy() for y in (y1, y2, y3)]
    got = rt.cpu().numpy()
    for ni, l in ((2, 3), (0, 0)):
        cols = []
        for k in range(2 * w.n2):
            e = np.zeros(w.shape, dtype=complex)
            e[k % w.n2, ni, l] = 1.0 if k < w.n2 else 1j
            out = curl_free_momentum(op, e)
            cols.append(np.concatenate([out[0][:, ni, l], out[1][:, ni, l], out[2][:, ni, l]]))
        A = np.array(cols).T
        Ar = np.vstack([A.real, A.imag])
        yc = np.concatenate([ys[0][:, ni, l], ys[1][:, ni, l], ys[2][:, ni, l]])
        g = Ar.T @ np.concatenate([yc.real, yc.imag])
        ref = g[:w.n2] + 1j * g[w.n2:]
        assert np.abs(got[:, ni, l] - ref).max() < 1e-10 * np.abs(ref).max(), (ni, l)


def test_fixed_point_iteration_gradient(torch):
    """The building blocks compose under autograd: one fixed-point iteration z_t -> L(z) z_t (eq. y_k,
    Section 4.3), written with the differentiable operators and torch's pointwise products (rho_t =
    f'(z) z_t on the grid, m^c, g . m^c with g = -grad z / rho, the Neumann projection), has a gradient
    (the adjoint chain: P_N^T, the transforms' transposes, m^c^T, E^T) that matches central differences
    on 16 random directions."""
    from paper_2206_09878_amd.autograd import evaluate, mc, project, to_physical, to_spectral
    from paper_2206_09878_amd.workloads import make_inputs
    p = plan_of(32, 33)
    w = p.w
    z = p.to_dev(make_inputs(w, seed=60, stage=0)["z"])
    k1 = torch.as_tensor(np.asarray(OPlan(oracle_config(w)).k1), device="cuda")
    k3 = torch.as_tensor(np.asarray(OPlan(oracle_config(w)).k3), device="cuda")
    with torch.no_grad():
        v0 = p.evaluate(0, z)
        zp = p.to_physical(v0)
        rho = w.rho_l * w.rho_h / (w.rho_h - (w.rho_h - w.rho_l) * zp)
        fp = rho * rho * (w.rho_h - w.rho_l) / (w.rho_l * w.rho_h)
        g1 = -p.to_physical((1j * k1)[None, None, :] * v0) / rho
        g2 = -p.to_physical(p.evaluate(1, z)) / rho
        g3 = -p.to_physical((1j * k3)[None, :, None] * v0) / rho
    W = crand(torch, w.shape, 61)

    def loss(zt):
        rt = project(p, 0, to_spectral(p, fp * to_physical(p, evaluate(p, 0, zt))))
        m1, m2, m3 = mc(p, rt)
        Lp = g1 * to_physical(p, evaluate(p, 0, m1)) + g2 * to_physical(p, evaluate(p, 0, m2, star=True)) \
            + g3 * to_physical(p, evaluate(p, 0, m3))
        out = project(p, 2, to_spectral(p, Lp))
        return torch.sum(torch.view_as_real(W) * torch.view_as_real(out))

    zt = crand(torch, w.shape, 62).requires_grad_(True)
    loss(zt).backward()
    grad = zt.grad.detach()
    eps = 1e-6
    with torch.no_grad():
        for k in range(16):
            d = crand(torch, w.shape, 200 + k)
            fd = (loss(zt + eps * d) - loss(zt - eps * d)).item() / (2 * eps)
            an = rdot(torch, grad, d)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (k, fd, an)


def test_rhs_gradient_through_the_operators(torch):
    """Steps 4 and 5 (RHS of phi2, eq. phi with the body force) written with the differentiable
    operators and torch's pointwise products: u = m/rho, T_ij = -m_i m_j/rho + tau_ij on the 3/2 grid,
    T_hat, N_i, RHS_phi2 = -k^2 N2 - d/dy(i k1 N1 + i k3 N3) + k^2 g rho, Dirichlet projection.  Its value
    equals lmvd_rhs (the native kernels) and its gradient in m1 matches central differences."""
    from paper_2206_09878_amd.autograd import evaluate, project, to_physical, to_spectral
    from paper_2206_09878_amd.workloads import make_inputs
    p = plan_of(32, 33)
    w = p.w
    op = OPlan(oracle_config(w))
    ik1 = torch.as_tensor(1j * np.asarray(op.k1), device="cuda")[None, None, :]
    ik3 = torch.as_tensor(1j * np.asarray(op.k3), device="cuda")[None, :, None]
    ksq = torch.as_tensor(np.asarray(op.ksq), device="cuda")[None]
    inp = make_inputs(w, seed=80, stage=0)
    z = p.to_dev(inp["z"])
    m1, m2, m3 = p.md(p.to_dev(inp["phi2"]), p.to_dev(inp["omega2"]), p.to_dev(inp["m1bar"]),
                      p.to_dev(inp["m3bar"]))
    mu, g = w.mu, w.g
    with torch.no_grad():
        zp = p.to_physical(p.evaluate(0, z))
        rho = w.rho_l * w.rho_h / (w.rho_h - (w.rho_h - w.rho_l) * zp)

    def rhs_phi(m1_):
        mp = [to_physical(p, evaluate(p, 0, m1_)), to_physical(p, evaluate(p, 0, m2, star=True)),
              to_physical(p, evaluate(p, 0, m3))]
        uh = [project(p, 0, to_spectral(p, x / rho)) for x in mp]
        d = []
        for ui in uh:
            v0 = evaluate(p, 0, ui)
            d.append([to_physical(p, ik1 * v0), to_physical(p, evaluate(p, 1, ui)), to_physical(p, ik3 * v0)])
        theta = d[0][0] + d[1][1] + d[2][2]
        Th = {}
        for i, j in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)):
            t = -mp[i] * mp[j] / rho + mu * (d[i][j] + d[j][i])
            if i == j:
                t = t - (2.0 / 3.0) * mu * theta
            Th[(i, j)] = Th[(j, i)] = project(p, 0, to_spectral(p, t))
        N = [ik1 * evaluate(p, 0, Th[(i, 0)]) + evaluate(p, 1, Th[(i, 1)]) + ik3 * evaluate(p, 0, Th[(i, 2)])
             for i in range(3)]
        dN = [ik1 * evaluate(p, 1, Th[(i, 0)]) + evaluate(p, 2, Th[(i, 1)]) + ik3 * evaluate(p, 1, Th[(i, 2)])
              for i in range(3)]
        R = -ksq * N[1] - (ik1 * dN[0] + ik3 * dN[2]) + ksq * g * to_spectral(p, rho)
        mask = torch.ones_like(R)
        mask[:, 0, 0] = 0.0
        return project(p, 1, R * mask)

    with torch.no_grad():
        native = p.rhs(z, m1, m2, m3)["phi2"]
        composed = rhs_phi(m1)
    torch.cuda.synchronize()
    err = (composed - native).abs().max().item() / native.abs().max().item()
    print("composed vs native RHS_phi2", err, flush=True)
    assert err < 1e-10
    W = crand(torch, w.shape, 81)
    loss = lambda x: torch.sum(torch.view_as_real(W) * torch.view_as_real(rhs_phi(x)))
    x = m1.clone().requires_grad_(True)
    loss(x).backward()
    grad = x.grad.detach()
    scale = m1.abs().max().item()
    eps = 1e-6 * scale
    with torch.no_grad():
        for k in range(16):
            dvec = crand(torch, w.shape, 300 + k)
            fd = (loss(m1 + eps * dvec) - loss(m1 - eps * dvec)).item() / (2 * eps)
            an = rdot(torch, grad, dvec)
            assert abs(fd - an) < 1e-5 * max(1.0, abs(an)), (k, fd, an)


def composed_substep(torch, p, op, st, hist, stage=0, prev=None):
    """One substep (Algorithm time_advanceDNS, in the oracle's order) written with the differentiable
    operators and torch's pointwise products; returns the new state, this stage's RHS and z_t.
    Stage ' takes prev = (RHS, z_t) of stage n."""
    from paper_2206_09878_amd.autograd import evaluate, mc, md, project, to_physical, to_spectral
    w = p.w
    ik1 = torch.as_tensor(1j * np.asarray(op.k1), device="cuda")[None, None, :]
    ik3 = torch.as_tensor(1j * np.asarray(op.k3), device="cuda")[None, :, None]
    ksq = torch.as_tensor(np.asarray(op.ksq), device="cuda")[None]
    phys = lambda v: to_physical(p, v)
    spec = lambda x: to_spectral(p, x)
    phi2, om2, z, m1bar, m3bar = st
    # 1. m^d
    md1, md2, md3 = md(p, phi2, om2, m1bar, m3bar)
    # 2. R_z and the fields fixed during the substep
    Vz = evaluate(p, 0, z)
    zp = phys(Vz)
    z1, z2, z3 = phys(ik1 * Vz), phys(evaluate(p, 1, z)), phys(ik3 * Vz)
    lap = phys(evaluate(p, 2, z) - ksq * Vz)
    rho = w.rho_l * w.rho_h / (w.rho_h - (w.rho_h - w.rho_l) * zp)
    fp = rho * rho * (w.rho_h - w.rho_l) / (w.rho_l * w.rho_h)
    mdp = [phys(evaluate(p, 0, md1)), phys(evaluate(p, 0, md2, star=True)), phys(evaluate(p, 0, md3))]
    Rz = project(p, 2, spec((-(mdp[0] * z1 + mdp[1] * z2 + mdp[2] * z3) + w.rhoD * lap) / rho))
    # BDF-like guess (eq. dzdt_guesses, beta^n = 0, beta' = -4): dt z_t = a . (z, h1, h2, h3)
    bp = w.beta_p
    a = (2.0, -2.0, 0.0, 0.0) if stage == 0 else (4.0 + bp, -(5.0 + 2.0 * bp), bp, 1.0)
    zt = (a[0] * z + a[1] * hist[0] + a[2] * hist[1] + a[3] * hist[2]) / w.dt

    def mc_of(zt_):
        return mc(p, project(p, 0, spec(fp * phys(evaluate(p, 0, zt_)))))

    # 3. fixed-point iterations
    for _ in range(w.kf):
        c1, c2, c3 = mc_of(zt)
        L = -(z1 * phys(evaluate(p, 0, c1)) + z2 * phys(evaluate(p, 0, c2, star=True))
              + z3 * phys(evaluate(p, 0, c3))) / rho
        zt = project(p, 2, spec(L)) + Rz
    c1, c2, c3 = mc_of(zt)
    m = [md1 + c1, md2 + c2, md3 + c3]
    # 4./5. fluxes and right-hand sides
    mp = [phys(evaluate(p, 0, m[0])), phys(evaluate(p, 0, m[1], star=True)), phys(evaluate(p, 0, m[2]))]
    uh = [project(p, 0, spec(x / rho)) for x in mp]
    d = []
    for ui in uh:
        v0 = evaluate(p, 0, ui)
        d.append([phys(ik1 * v0), phys(evaluate(p, 1, ui)), phys(ik3 * v0)])
    theta = d[0][0] + d[1][1] + d[2][2]
    Th = {}
    for i, j in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)):
        t = -mp[i] * mp[j] / rho + w.mu * (d[i][j] + d[j][i])
        if i == j:
            t = t - (2.0 / 3.0) * w.mu * theta
        Th[(i, j)] = Th[(j, i)] = project(p, 0, spec(t))
    N = [ik1 * evaluate(p, 0, Th[(i, 0)]) + evaluate(p, 1, Th[(i, 1)]) + ik3 * evaluate(p, 0, Th[(i, 2)])
         for i in range(3)]
    dN = [ik1 * evaluate(p, 1, Th[(i, 0)]) + evaluate(p, 2, Th[(i, 1)]) + ik3 * evaluate(p, 1, Th[(i, 2)])
          for i in range(3)]
    mask = torch.ones_like(Vz)
    mask[:, 0, 0] = 0.0
    R_phi = project(p, 1, mask * (-ksq * N[1] - (ik1 * dN[0] + ik3 * dN[2]) + ksq * w.g * spec(rho)))
    R_om = project(p, 1, mask * (ik3 * N[0] - ik1 * N[2]))
    col = 1.0 - mask                                  # the (0,0) column alone

    def mean_rhs(T):
        return project(p, 2, col * evaluate(p, 1, T).real.to(Vz.dtype))[:, 0, 0].real

    R1, R3 = mean_rhs(Th[(0, 1)]), mean_rhs(Th[(2, 1)])
    R = dict(phi2=R_phi, omega2=R_om, m1bar=R1, m3bar=R3)
    X = dict(phi2=phi2, omega2=om2, m1bar=m1bar, m3bar=m3bar)
    if stage == 0:
        out = {k: X[k] + 0.5 * w.dt * R[k] for k in X}
        out["z"] = z + 0.5 * w.dt * zt
    else:
        Rp, ztp = prev
        out = {k: X[k] + w.dt * (R[k] - 0.5 * Rp[k]) for k in X}
        out["z"] = z + w.dt * (zt - 0.5 * ztp)
    out["zt"] = zt
    out["rhs"] = R
    return out


def test_substep_gradient_through_the_operators(torch):
    """The whole stage-n substep composed from the differentiable operators equals lmvd_substep (the
    native kernels) on every output, and the gradient of a real objective of its outputs with respect
    to the input z (through rho(z), R_z, the guess, the fixed point, m^c, the fluxes and RK2) matches
    Richardson-extrapolated central differences on 16 random directions."""
    from paper_2206_09878_amd.workloads import make_inputs
    p = plan_of(32, 33)
    w = p.w
    op = OPlan(oracle_config(w))
    inp = make_inputs(w, seed=90, stage=0)
    st = [p.to_dev(inp[k]) for k in ("phi2", "omega2", "z", "m1bar", "m3bar")]
    hist = [p.to_dev(h) for h in inp["hist"]]
    with torch.no_grad():
        ref = composed_substep(torch, p, op, st, hist)
    # the native substep from the same inputs
    d = [x.clone() for x in st]
    z_out, zt = p.empty(), p.empty()
    rhs = {"phi2": p.empty(), "omega2": p.empty(),
           "m1bar": torch.empty(w.n2, dtype=torch.float64, device="cuda"),
           "m3bar": torch.empty(w.n2, dtype=torch.float64, device="cuda")}
    p.substep(0, d[0], d[1], d[2], d[3], d[4], z_out=z_out, hist=hist, rhs_out=rhs, zt_out=zt)
    torch.cuda.synchronize()
    native = dict(phi2=d[0], omega2=d[1], z=z_out, m1bar=d[3], m3bar=d[4], zt=zt)
    for k, v in native.items():
        e = (ref[k] - v).abs().max().item() / max(v.abs().max().item(), 1e-300)
        print("composed vs native", k, e, flush=True)
        assert e < 1e-9, (k, e)
    W = {k: (crand(torch, w.shape, 91 + i) if k in ("z", "phi2", "omega2") else
             torch.randn(w.n2, dtype=torch.float64, device="cuda")) for i, k in enumerate(("z", "phi2", "omega2",
                                                                                         "m1bar", "m3bar"))}

    def loss(z):
        out = composed_substep(torch, p, op, [st[0], st[1], z, st[3], st[4]], hist)
        tot = 0.0
        for k, wk in W.items():
            o = out[k]
            tot = tot + (torch.sum(torch.view_as_real(wk) * torch.view_as_real(o)) if o.is_complex()
                         else torch.sum(wk * o))
        return tot

    z0 = st[2].clone().requires_grad_(True)
    loss(z0).backward()
    grad = z0.grad.detach()
    # central differences at eps and eps/2, Richardson-extrapolated: the objective has large third
    # derivatives (the guess carries 1/dt), so plain central differences carry a visible O(eps^2) term
    eps = 1e-6 * st[2].abs().max().item()
    with torch.no_grad():
        for k in range(16):
            dvec = crand(torch, w.shape, 400 + k)
            c = lambda e: (loss(st[2] + e * dvec) - loss(st[2] - e * dvec)).item() / (2 * e)
            f1, f2 = c(eps), c(0.5 * eps)
            fd = (4.0 * f2 - f1) / 3.0
            an = rdot(torch, grad, dvec)
            print("direction", k, "central", f1, "extrapolated", fd, "adjoint", an, flush=True)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (k, f1, fd, an)


def test_multistep_gradient_with_checkpoints(torch):
    """The adjoint workload's pattern at 32 x 33 x 32: 4 RK steps (8 substeps, stages n and ' with
    the z history ring) composed from the differentiable operators, checkpointed every 2 RK steps
    (torch.utils.checkpoint recomputes each segment's forward in the backward pass); objective the
    kinetic energy of m^d at the final time, (1/2) mean |m^d|^2 / rho on the 3/2 grid; gradient with
    respect to the initial z.  The checkpointed gradient equals the one kept in memory, and matches
    Richardson-extrapolated central differences on 4 random directions."""
    from torch.utils.checkpoint import checkpoint

    from paper_2206_09878_amd.autograd import evaluate, md, to_physical
    from paper_2206_09878_amd.workloads import make_inputs
    p = plan_of(32, 33)
    w = p.w
    op = OPlan(oracle_config(w))
    inp = make_inputs(w, seed=95, stage=0)
    st0 = [p.to_dev(inp[k]) for k in ("phi2", "omega2", "z", "m1bar", "m3bar")]
    hist0 = [p.to_dev(h) for h in inp["hist"]]

    def rk_step(phi2, om2, z, m1bar, m3bar, h1, h2, h3):
        a = composed_substep(torch, p, op, [phi2, om2, z, m1bar, m3bar], [h1, h2, h3], stage=0)
        zp = a["z"]
        b = composed_substep(torch, p, op, [a["phi2"], a["omega2"], zp, a["m1bar"], a["m3bar"]], [z, h1, h2],
                             stage=1, prev=(a["rhs"], a["zt"]))
        # history for the next stage n: z^{n,'}, z^n, z^{n-1,'}
        return b["phi2"], b["omega2"], b["z"], b["m1bar"], b["m3bar"], zp, z, h1

    def objective(z0, ckpt):
        carry = (st0[0], st0[1], z0, st0[3], st0[4], *hist0)
        for seg in range(2):
            def segment(*c):
                for _ in range(2):
                    c = rk_step(*c)
                return c
            carry = checkpoint(segment, *carry, use_reentrant=False) if ckpt else segment(*carry)
        phi2, om2, z, m1bar, m3bar = carry[:5]
        m1, m2, m3 = md(p, phi2, om2, m1bar, m3bar)
        zp = to_physical(p, evaluate(p, 0, z))
        rho = w.rho_l * w.rho_h / (w.rho_h - (w.rho_h - w.rho_l) * zp)
        ke = sum(to_physical(p, evaluate(p, 0, m, star=(i == 1))) ** 2 for i, m in enumerate((m1, m2, m3)))
        return 0.5 * torch.mean(ke / rho)

    grads = []
    for ckpt in (True, False):
        z0 = st0[2].clone().requires_grad_(True)
        objective(z0, ckpt).backward()
        grads.append(z0.grad.detach())
    diff = (grads[0] - grads[1]).abs().max().item() / grads[1].abs().max().item()
    print("checkpointed vs stored gradient", diff, flush=True)
    assert diff < 1e-12
    eps = 1e-6 * st0[2].abs().max().item()
    with torch.no_grad():
        for k in range(4):
            dvec = crand(torch, w.shape, 500 + k)
            c = lambda e: (objective(st0[2] + e * dvec, False) - objective(st0[2] - e * dvec, False)).item() / (2 * e)
            f1, f2 = c(eps), c(0.5 * eps)
            fd = (4.0 * f2 - f1) / 3.0
            an = rdot(torch, grads[0], dvec)
            print("direction", k, "central", f1, "extrapolated", fd, "adjoint", an, flush=True)
            assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12 * abs(f1) + 1e-300), (k, f1, fd, an)
