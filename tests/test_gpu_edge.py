"""Degenerate cases and the smallest grids, GPU against the oracle (1e-11):

  * constant density (rho_l = rho_h): f' = 0, so m^c = 0 and L = 0; the
    substep reduces to the incompressible method (its oracle reduction is
    pinned in tests/test_oracle_substep.py);
  * a state that is a mean z profile only (no momentum, no fluctuation): every
    momentum output and the fluctuating RHS are exactly zero, and z_t is
    the diffusion of the profile;
  * the smallest grids the plans accept in this family: 8 x 9 x 8 (M = 12,
    generic transforms, n2 one above the order), 16 x 9 x 16, and N1 != N3.
"""
import dataclasses

import numpy as np
import pytest

from paper_2206_09878_amd.workloads import make_inputs, workload
from tests.test_gpu_parity import check_pair, rhs_tolerances, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.mark.parametrize("stage", [0, 1])
def test_constant_density(torch, stage):
    w = dataclasses.replace(workload("small", n=16, n2=25), rho_l=2.0, rho_h=2.0)
    print("constant density", (w.n1, w.n2, w.n3), "stage", stage, flush=True)
    got, ref = run_pair(w, stage, seed=70)
    for x in got["mc"]:
        assert np.abs(x).max() < 1e-14 * max(1.0, np.abs(got["md"][0]).max())
    check_pair(got, ref)


def test_mean_profile_only(torch):
    w = workload("small", n=16, n2=25)
    inp = make_inputs(w, seed=71, stage=0)
    z = np.zeros_like(inp["z"])
    z[:, 0, 0] = inp["z"][:, 0, 0].real
    zero = np.zeros_like(z)
    inputs = dict(phi2=zero, omega2=zero.copy(), z=z, m1bar=np.zeros(w.n2), m3bar=np.zeros(w.n2),
                  hist=[z.copy(), z.copy(), z.copy()])
    got, ref = run_pair(w, 0, inputs=inputs)
    for k in ("phi2", "omega2"):
        assert np.abs(got["rhs"][k]).max() == 0.0 and np.abs(ref["rhs"][k]).max() == 0.0
    assert np.abs(got["zt"][:, 1:, :]).max() == 0.0 and np.abs(got["zt"][:, 0, 1:]).max() == 0.0
    check_pair(got, ref)


@pytest.mark.parametrize("n1,n3,n2", [(8, 8, 9), (16, 16, 9), (16, 24, 17), (24, 16, 17)])
def test_smallest_grids(torch, n1, n3, n2):
    w = workload("small", n=n1, n2=n2)
    if n3 != n1:
        w = dataclasses.replace(w, n3=n3, m3=3 * n3 // 2)
    print("grid", (w.n1, w.n2, w.n3), (w.m1, w.m3), flush=True)
    got, ref = run_pair(w, 0, seed=72)
    check_pair(got, ref, rhs_tol=rhs_tolerances(w, 0, 72, ref=ref))
