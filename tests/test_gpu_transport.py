"""Variable transport coefficients, mu = g(z) and rho D_z = q(z) or f(z) q(z)
(Section 2), on the GPU path against the oracle, through the C ABI.

The oracle's variable-coefficient terms are pinned in
tests/test_oracle_transport.py.  Here one substep of the HIP path is compared
with it element by element (1e-11, the RHS fields within 4x the oracle's own
FFT-rounding spread where that is larger), on:

  * the register x-pass with all planes in one batch (z kept in its zbuf slot
    for the mu(z) S_ij pass; filtered fixed-point iterates), stages n and ';
  * the register x-pass with plane batches (z transformed again);
  * the generic x-pass (M = 36) with ragged plane batches;
  * a mid size (64 x 65 x 64, M = 96);
  * row counts n2 = 14 and 19 (16 x n2 x 16), whose unrolled column sweeps end in longer tails;
  * each law alone (only mu(z), only rho D(z), both forms of rho D);
  * the grouped HIP graph of two such instances, equal to eager substeps bit
    for bit.
"""
import dataclasses

import pytest

from paper_2206_09878_amd.workloads import make_inputs, workload
from tests.test_gpu_parity import check_pair, rhs_tolerances, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def with_laws(w, mu=True, rhod=True, form=1):
    """mu(z) = mu (1 + 0.5 z - 0.3 z^2 + 0.2 z^3); q(z) = rhoD (1 + 0.4 z + 0.1 z^2 - 0.05 z^3)."""
    kw = {}
    if mu:
        kw["mu_z"] = (0.5 * w.mu, -0.3 * w.mu, 0.2 * w.mu)
    if rhod:
        kw["rhoD_z"] = (0.4 * w.rhoD, 0.1 * w.rhoD, -0.05 * w.rhoD)
        kw["rhoD_form"] = form
    return dataclasses.replace(w, **kw)


def check(w, stage, seed, plane_batch=0):
    print("transport", w.name, (w.n1, w.n2, w.n3), "mu_z", w.mu_z, "rhoD_z", w.rhoD_z, "form", w.rhoD_form,
          "stage", stage, "plane_batch", plane_batch, flush=True)
    got, ref = run_pair(w, stage, seed=seed, plane_batch=plane_batch)
    return check_pair(got, ref, rhs_tol=rhs_tolerances(w, stage, seed, ref=ref))


@pytest.mark.parametrize("stage", [0, 1])
def test_variable_transport_register_path(torch, stage):
    check(with_laws(workload("small")), stage, seed=21)


def test_variable_transport_register_path_plane_batches(torch):
    check(with_laws(workload("small")), 0, seed=22, plane_batch=8)


def test_variable_transport_generic_path_ragged_batches(torch):
    w = workload("small", n=24, n2=33)       # M = 36: the generic x-pass
    check(with_laws(w), 1, seed=23, plane_batch=7)


def test_variable_transport_mid_size(torch):
    check(with_laws(workload("mixing128", n=64, n2=65)), 0, seed=24)


@pytest.mark.parametrize("n2,stage", [(14, 1), (19, 0)])
def test_variable_transport_row_counts(torch, n2, stage):
    check(with_laws(workload("small", n=16, n2=n2)), stage, seed=25 + n2)


@pytest.mark.parametrize("mu,rhod,form", [(True, False, 0), (False, True, 0), (False, True, 1)])
def test_each_transport_law_alone(torch, mu, rhod, form):
    check(with_laws(workload("small", n=16, n2=25), mu, rhod, form), 0, seed=25)


def test_variable_transport_differs_from_constant(torch):
    """The laws reach the result: the same inputs with constant mu, rho D give
    another state (guards against a path that ignores the coefficients)."""
    from tests.test_gpu_parity import rel
    w = workload("small", n=16, n2=25)
    got_v, _ = run_pair(with_laws(w), 0, seed=26)
    got_c, _ = run_pair(w, 0, seed=26)
    assert rel(got_v["rhs"]["phi2"], got_c["rhs"]["phi2"]) > 1e-6
    assert rel(got_v["zt"], got_c["zt"]) > 1e-6


def test_variable_transport_in_a_grouped_graph(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    ws = [with_laws(workload("small")), with_laws(workload("small", n=48, n2=49))]   # M = 48, 72
    mk = lambda: [Stepper(Plan(w), make_inputs(w, seed=30 + i, stage=0), stage=0) for i, w in enumerate(ws)]
    A, B = mk(), mk()
    g = GraphBatch(A, nsub=4)
    assert g.grouped
    for launch in range(2):
        for s in B:
            for _ in range(4):
                s.substep()
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip(A, B):
            sa, sb = a.state(), b.state()
            for k in ("z", "phi2", "omega2", "m1bar", "m3bar"):
                assert torch.equal(sa[k], sb[k]), (launch, k)
