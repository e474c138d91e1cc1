"""GPU parity: the HIP library against the oracle, element by element, on the
same seeded inputs.  Bar: relative max-norm difference per field <= 1e-11.

Every call goes through the C ABI (ctypes binding)."""
import numpy as np
import pytest

from oracle.fourier import to_physical, to_spectral
from oracle.lmvd import Plan as OPlan, apply, curl_free_momentum, divergence_free_momentum, substep
from paper_2206_09878_amd.workloads import make_inputs, workload
from tests.conftest import oracle_config

pytestmark = pytest.mark.gpu
TOL = 1e-11


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def gplan(w, **kw):
    from paper_2206_09878_amd.lmvd import Plan
    return Plan(w, **kw)


def host(t):
    return t.detach().cpu().numpy()


def hermitian(rng, shape):
    V = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nn = shape[1]
    for ni in range(1, (nn + 1) // 2):
        V[:, nn - ni, 0] = np.conj(V[:, ni, 0])
    V[:, 0, 0] = V[:, 0, 0].real
    return V


GRIDS = [("small", None, None), ("small", 48, 17), ("small", 64, 33), ("mixing128", 128, 17),
         ("rt512", 512, 9)]


@pytest.mark.parametrize("name,n,n2", GRIDS)
def test_transforms(torch, name, n, n2):
    w = workload(name, n=n, n2=n2)
    p = gplan(w)
    rng = np.random.default_rng(1)
    V = hermitian(rng, w.shape)
    ref = to_physical(V, w.m1, w.m3)
    got = host(p.to_physical(p.to_dev(V)))
    u = rng.standard_normal((w.n2, w.m3, w.m1))
    refV = to_spectral(u, w.n1, w.n3)
    gotV = host(p.to_spectral(p.to_dev(u)))
    print(f"transforms {w.m1}x{w.m3}: inverse {rel(got, ref):.1e}, forward {rel(gotV, refV):.1e}", flush=True)
    assert rel(got, ref) < TOL
    assert rel(gotV, refV) < TOL


@pytest.mark.parametrize("name,n,n2", [("small", None, None), ("small", 48, 49), ("small", 16, 14), ("small", 16, 19)])
def test_evaluate_and_project(torch, name, n, n2):
    w = workload(name, n=n, n2=n2)
    p = gplan(w)
    op = OPlan(oracle_config(w))
    rng = np.random.default_rng(2)
    C = hermitian(rng, w.shape)
    Cs = hermitian(rng, w.shape_star)
    for d in range(3):
        assert rel(host(p.evaluate(d, p.to_dev(C))), apply(op.sp.E[d], C)) < TOL
    assert rel(host(p.evaluate(0, p.to_dev(Cs), star=True)), apply(op.sp.F[0], Cs)) < TOL
    for kind, name_ in enumerate(("plain", "dirichlet", "neumann")):
        assert rel(host(p.project(kind, p.to_dev(C))), op.project(C, name_)) < TOL


@pytest.mark.parametrize("name,n,n2", [("small", None, None), ("small", 48, 49), ("mixing128", 64, 65)])
def test_md_mc(torch, name, n, n2):
    w = workload(name, n=n, n2=n2)
    p = gplan(w)
    op = OPlan(oracle_config(w))
    inp = make_inputs(w, seed=3)
    ref = divergence_free_momentum(op, inp["phi2"], inp["omega2"], inp["m1bar"], inp["m3bar"])
    got = p.md(p.to_dev(inp["phi2"]), p.to_dev(inp["omega2"]), p.to_dev(inp["m1bar"]), p.to_dev(inp["m3bar"]))
    for g, r in zip(got, ref):
        assert rel(host(g), r) < TOL
    rng = np.random.default_rng(4)
    rhot = hermitian(rng, w.shape)
    ref = curl_free_momentum(op, rhot)
    got = p.mc(p.to_dev(rhot))
    for g, r in zip(got, ref[:3]):
        assert rel(host(g), r) < TOL


def oracle_substep(w, stage, inp, kf=None, guess_mode=0):
    """The oracle's substep (with diagnostics) from the inputs of make_inputs' form."""
    op = OPlan(oracle_config(w))
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    kw = {}
    if stage == 1:
        kw = dict(rhs_prev=inp["rhs_prev"], zt_prev=inp["zt_prev"])
    return substep(op, st, stage, hist=inp["hist"], kf=kf, guess="zero" if guess_mode else "bdf",
                   diagnostics=True, **kw)


def gpu_substep(w, stage, inp, kf=None, guess_mode=0, plane_batch=0, tile=0):
    """The same substep through lmvd_substep, with the m^d and m^c diagnostics; host copies."""
    import torch
    p = gplan(w, plane_batch=plane_batch)
    if tile:
        assert p.autotune(force=tile)[0] == tile
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    d = {k: p.to_dev(v) for k, v in st.items()}
    hist = [p.to_dev(h) for h in inp["hist"]]
    z_out = p.empty()
    rhs = {"phi2": p.empty(), "omega2": p.empty(),
           "m1bar": torch.empty(w.n2, dtype=torch.float64, device="cuda"),
           "m3bar": torch.empty(w.n2, dtype=torch.float64, device="cuda")}
    zt = p.empty()
    md = [p.empty(), p.empty(True), p.empty()]
    mc = [p.empty(), p.empty(True), p.empty()]
    args = dict(z_out=z_out, hist=hist, kf=-1 if kf is None else kf, guess_mode=guess_mode, rhs_out=rhs,
                zt_out=zt, md=md, mc=mc)
    if stage == 1:
        args["rhs_prev"] = {k: p.to_dev(v) for k, v in inp["rhs_prev"].items()}
        args["zt_prev"] = p.to_dev(inp["zt_prev"])
    p.substep(stage, d["phi2"], d["omega2"], d["z"], d["m1bar"], d["m3bar"], **args)
    torch.cuda.synchronize()
    return dict(phi2=host(d["phi2"]), omega2=host(d["omega2"]), z=host(z_out), m1bar=host(d["m1bar"]),
                m3bar=host(d["m3bar"]), zt=host(zt), rhs={k: host(v) for k, v in rhs.items()},
                md=[host(x) for x in md], mc=[host(x) for x in mc])


def run_pair(w, stage, seed=0, kf=None, guess_mode=0, plane_batch=0, tile=0, inputs=None):
    """One substep on the GPU and in the oracle from the same inputs (tile: force the z tile divisor;
    inputs: a dict like make_inputs' instead of the seeded one)."""
    inp = make_inputs(w, seed=seed, stage=stage) if inputs is None else inputs
    ref = oracle_substep(w, stage, inp, kf=kf, guess_mode=guess_mode)
    got = gpu_substep(w, stage, inp, kf=kf, guess_mode=guess_mode, plane_batch=plane_batch, tile=tile)
    return got, ref


class scipy_fft_in_oracle:
    """Run the oracle with scipy.fft in place of numpy.fft: the same sums with
    a different rounding."""

    def __enter__(self):
        import types
        import scipy.fft as sf
        import oracle.fourier as F
        self.F, self.np = F, F.np
        shim = types.SimpleNamespace(**{k: getattr(np, k) for k in dir(np) if not k.startswith("__")})
        shim.fft = types.SimpleNamespace(ifft2=lambda x, axes: sf.ifft2(x, axes=axes),
                                         fft2=lambda x, axes: sf.fft2(x, axes=axes))
        F.np = shim
        return self

    def __exit__(self, *exc):
        self.F.np = self.np


class dense_solves_in_oracle:
    """Run the oracle with its banded solves done as dense pivoted LU (numpy.linalg.solve), eliminating
    from the first row (reverse = False) or, on the row- and column-reversed system, from the last row:
    the same systems with other elimination orders and rounding."""

    def __init__(self, reverse=False):
        self.reverse = reverse

    def __enter__(self):
        import oracle.lmvd as O
        self.O, self.orig = O, O.banded_solve
        rev = self.reverse

        def dense(A, B):
            shp = B.shape
            b = B.reshape(shp[0], -1)
            if rev:
                return np.linalg.solve(A[::-1, ::-1], b[::-1])[::-1].reshape(shp)
            return np.linalg.solve(A, b).reshape(shp)
        O.banded_solve = dense
        return self

    def __exit__(self, *exc):
        self.O.banded_solve = self.orig


class transform_rounding_in_oracle:
    """Run the oracle with one unit of float64 rounding, at the scale of each transform's largest output,
    added to every output of its inverse and forward transforms (seeded uniform noise): a model of the
    rounding that another transform implementation makes."""

    def __init__(self, seed=77):
        self.rng = np.random.default_rng(seed)

    def __enter__(self):
        import oracle.adjoint as A
        import oracle.lmvd as O
        self.mods = [(M, M.to_physical, M.to_spectral) for M in (O, A)]
        eps = 2.0 ** -53

        def noisy(f):
            def g(*a):
                y = f(*a)
                s = eps * np.abs(y).max()
                if np.iscomplexobj(y):
                    return y + s * (self.rng.uniform(-1, 1, y.shape) + 1j * self.rng.uniform(-1, 1, y.shape))
                return y + s * self.rng.uniform(-1, 1, y.shape)
            return g
        for M, inv, fwd in self.mods:
            M.to_physical, M.to_spectral = noisy(inv), noisy(fwd)
        return self

    def __exit__(self, *exc):
        for M, inv, fwd in self.mods:
            M.to_physical, M.to_spectral = inv, fwd


def output_errors(got, ref):
    """Relative max-norm difference of every output of a substep (state, z_t, RHS, m^d, m^c)."""
    errs = {}
    for k in ("phi2", "omega2", "z", "m1bar", "m3bar"):
        errs[k] = rel(got[k], ref["state"][k])
    errs["zt"] = rel(got["zt"], ref["zt"])
    for k in ("phi2", "omega2", "m1bar", "m3bar"):
        errs["rhs_" + k] = rel(got["rhs"][k], ref["rhs"][k])
    if "md" in got:
        for i in range(3):
            errs[f"md{i}"] = rel(got["md"][i], ref["diag"]["md"][i])
            errs[f"mc{i}"] = rel(got["mc"][i], ref["diag"]["mc"][i])
    return errs


def spread_tolerances(w, stage, ref, inputs, kf=None, rounding=False, factor=4.0):
    """Per-output bound: 1e-11, or `factor` times the oracle's own spread where the output amplifies
    float64 rounding more than that (derivatives of fields with large plane means, small differences of
    large terms).  The spread is the difference between the oracle and the oracle run with scipy's FFT
    in place of numpy's; with rounding, also with dense pivoted solves in place of the banded ones and
    one unit of rounding, at the scale of each transform's largest output, added to every transform
    output: the change that the rounding of another implementation of the same arithmetic makes to
    the output."""
    inp = inputs
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    kw = dict(rhs_prev=inp["rhs_prev"], zt_prev=inp["zt_prev"]) if stage == 1 else {}
    import contextlib
    with scipy_fft_in_oracle(), (dense_solves_in_oracle() if rounding else contextlib.nullcontext()), \
            (transform_rounding_in_oracle() if rounding else contextlib.nullcontext()):
        alt = substep(OPlan(oracle_config(w)), st, stage, hist=inp["hist"], kf=kf, diagnostics=True, **kw)
    alt_out = dict(alt["state"], zt=alt["zt"], rhs=alt["rhs"], md=alt["diag"]["md"], mc=alt["diag"]["mc"])
    return {k: max(TOL, factor * v) for k, v in output_errors(alt_out, ref).items()}


def rhs_tolerances(w, stage, seed, kf=None, ref=None, inputs=None):
    """The spread bounds of the stage RHS outputs (see spread_tolerances), keyed phi2, omega2, m1bar, m3bar."""
    inp = make_inputs(w, seed=seed, stage=stage) if inputs is None else inputs
    t = spread_tolerances(w, stage, ref, inp, kf=kf)
    return {k[4:]: v for k, v in t.items() if k.startswith("rhs_")}


def check_pair(got, ref, tol=TOL, rhs_tol=None, tols=None):
    errs = output_errors(got, ref)
    bounds = {k: tol for k in errs}
    if rhs_tol:
        for k, v in rhs_tol.items():
            bounds["rhs_" + k] = v
    if tols:
        bounds.update({k: v for k, v in tols.items() if k in bounds})
    print("  " + ", ".join(f"{k} {v:.1e}/{bounds[k]:.0e}" for k, v in errs.items()), flush=True)
    bad = {k: (v, bounds[k]) for k, v in errs.items() if not v < bounds[k]}
    assert not bad, (bad, errs)
    return errs


@pytest.mark.parametrize("stage", [0, 1])
def test_substep_small(torch, stage):
    w = workload("small")
    got, ref = run_pair(w, stage)
    check_pair(got, ref)


# Row counts of every residue mod 8: the column sweeps run their rows (n2, or n2 + 1 for the B* sweeps)
# in unrolled blocks of 4 or 8 steps and then a tail of the remaining steps.
ROWS = [12, 13, 14, 15, 16, 18, 19, 20, 22]


@pytest.mark.parametrize("n2", ROWS)
@pytest.mark.parametrize("stage", [0, 1])
def test_substep_row_counts(torch, n2, stage):
    w = workload("small", n=16, n2=n2)
    got, ref = run_pair(w, stage, seed=40 + n2)
    check_pair(got, ref)


@pytest.mark.parametrize("kf,guess_mode", [(0, 0), (1, 0), (3, 1)])
def test_substep_iteration_counts(torch, kf, guess_mode):
    w = workload("small", n=16, n2=25)
    got, ref = run_pair(w, 0, seed=5, kf=kf, guess_mode=guess_mode)
    check_pair(got, ref)


def test_substep_ragged_plane_batches(torch):
    w = workload("small", n=24, n2=33)       # M = 36: radices 2, 3, 3 / 2, 9
    got, ref = run_pair(w, 1, seed=6, plane_batch=7)
    check_pair(got, ref)


@pytest.mark.parametrize("name,n,n2", [("mixing128", 64, 65), ("adjoint96", 96, 97)])
def test_substep_mid(torch, name, n, n2):
    w = workload(name, n=n, n2=n2)
    got, ref = run_pair(w, 0, seed=7)
    check_pair(got, ref, rhs_tol=rhs_tolerances(w, 0, 7, ref=ref))


def test_substep_mixing_layer_full_size(torch):
    """The mixing-layer configuration at its full size, 128x129x128 on the
    192 x 192 grid (density 1 -> 7, broadband perturbation, mean shear), one
    stage-n substep against the oracle."""
    w = workload("mixing128")
    print("mixing128 full size", (w.n1, w.n2, w.n3), flush=True)
    got, ref = run_pair(w, 0, seed=1)
    check_pair(got, ref, rhs_tol=rhs_tolerances(w, 0, 1, ref=ref))


@pytest.mark.parametrize("name,n,n2,laws", [("small", None, None, False), ("small", 24, 33, True),
                                             ("mixing128", 64, 65, False)])
def test_rhs_entry_point(torch, name, n, n2, laws):
    """lmvd_rhs (steps 4 and 5 alone) from the oracle's own z and m = m^d + m^c
    of a substep, against that substep's RHS: row a9 in isolation.  The 36-point
    case runs the generic x-pass with variable transport laws."""
    import dataclasses
    w = workload(name, n=n, n2=n2)
    if laws:
        w = dataclasses.replace(w, mu_z=(0.5 * w.mu, -0.3 * w.mu, 0.2 * w.mu),
                                rhoD_z=(0.4 * w.rhoD, 0.0, 0.0), rhoD_form=1)
    print("lmvd_rhs", name, (w.n1, w.n2, w.n3), "laws", laws, flush=True)
    inp = make_inputs(w, seed=8, stage=0)
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    ref = substep(OPlan(oracle_config(w)), st, 0, hist=inp["hist"], diagnostics=True)
    md, mc = ref["diag"]["md"], ref["diag"]["mc"]
    p = gplan(w)
    got = p.rhs(p.to_dev(st["z"]), *[p.to_dev(md[i] + mc[i]) for i in range(3)])
    torch.cuda.synchronize()
    tol = rhs_tolerances(w, 0, 8, ref=ref)
    for k in ("phi2", "omega2", "m1bar", "m3bar"):
        e = rel(host(got[k]), ref["rhs"][k])
        assert e < tol[k], (k, e, tol[k])


def test_trajectory_three_substeps_small(torch):
    """Config 0 trajectory: substeps n, ', n, each side free-running on its own
    outputs (history rotation, stored RHS and z_t between the stages), from the
    same seeded state and synthetic history; every state field within 1e-11."""
    from oracle.lmvd import Integrator
    from paper_2206_09878_amd.lmvd import Stepper
    w = workload("small")
    p = gplan(w)
    op = OPlan(oracle_config(w))
    inp = make_inputs(w, seed=0, stage=0)
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    it = Integrator(op, st, hist=inp["hist"])
    it.step()                                   # substeps n and '
    ref = substep(op, it.state, 0, hist=it.hist)["state"]   # substep n of the next step
    s = Stepper(p, inp, stage=0)
    for _ in range(3):
        s.substep()
    torch.cuda.synchronize()
    got = dict(phi2=host(s.phi2), omega2=host(s.omega2), z=host(s.z), m1bar=host(s.m1bar), m3bar=host(s.m3bar))
    errs = {k: rel(got[k], ref[k]) for k in got}
    assert all(v < TOL for v in errs.values()), errs


def test_trajectory_drift_curve_small(torch):
    """Config 0 drift curve: 20 RK steps (40 substeps), each side free-running on its own outputs from
    the same seeded state and synthetic history.  After every step the relative max-norm difference of
    each state field is printed; the first step is within 1e-11, and the whole curve within 1e-10 (a
    bound on the growth of the two implementations' rounding along the trajectory)."""
    from oracle.lmvd import Integrator
    from paper_2206_09878_amd.lmvd import Stepper
    w = workload("small")
    p = gplan(w)
    op = OPlan(oracle_config(w))
    inp = make_inputs(w, seed=0, stage=0)
    st = {k: inp[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    it = Integrator(op, st, hist=inp["hist"])
    s = Stepper(p, inp, stage=0)
    curve = []
    for step in range(20):
        ref = it.step()
        s.substep()
        s.substep()
        torch.cuda.synchronize()
        got = dict(phi2=host(s.phi2), omega2=host(s.omega2), z=host(s.z), m1bar=host(s.m1bar), m3bar=host(s.m3bar))
        errs = {k: rel(got[k], ref[k]) for k in got}
        curve.append(max(errs.values()))
        print(f"step {step + 1:2d}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    assert curve[0] < TOL, curve
    assert max(curve) < 1e-10, curve


@pytest.mark.parametrize("plane_batch", [0, 64])
def test_filtered_and_spectral_iterates_against_oracle(torch, plane_batch):
    """64x65x64, stage ': all planes in one batch (the fixed-point iterates before the last are
    z-filtered on the 3/2 grid, wall planes from the Neumann projection's wall-row weights) and a plane
    batch of n2 - 1 (the spectral path: forward transform, projection, values, inverse transform), each
    against the oracle.  The 768-point filter kernel is covered the same way at 512 x 17 x 512."""
    w = workload("mixing128", n=64, n2=65)
    got, ref = run_pair(w, 1, seed=9, plane_batch=plane_batch)
    check_pair(got, ref, rhs_tol=rhs_tolerances(w, 1, 9, ref=ref))
