"""The linear-stability tool (paper_2206_09878_amd.stability, Section 3.3.2,
Appendix B) against the oracle's step matrix (built by running the scheme on
unit history vectors) and against closed forms:

  * zero stability with beta' = -4: eigenvalues {1, lambda1^k, lambda1^k, 0},
    region = the open unit disc for every k;
  * lambda1 = 0: one iteration is exact, the physical eigenvalue is the RK2
    polynomial 1 + h + h^2/2 and the region is the RK2 region;
  * converged iterations: the RK2 polynomial of h = dt lambda2 / (1 - lambda1);
  * constants are preserved for any beta^n, beta';
  * beta' = -1 loses zero stability inside the unit disc.
"""
import numpy as np
import pytest

import oracle.ode_model as om
from paper_2206_09878_amd import stability as st


@pytest.mark.parametrize("k", [1, 2, 4])
def test_step_matrix_equals_the_oracle(k):
    rng = np.random.default_rng(k)
    for _ in range(20):
        lam1 = complex(*rng.uniform(-0.9, 0.9, 2))
        lam2 = complex(*rng.uniform(-2.0, 0.5, 2))
        for bp in (-4.0, -1.0, 0.5):
            A = st.step_matrix(lam1, lam2, k, beta_p=bp)
            B = om.linear_step_matrix(lam1, lam2, k, beta_p=bp)
            assert np.abs(A - B).max() < 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_zero_stability_is_the_unit_disc(k):
    lam1 = np.array([0.7 + 0.25j, 0.5j, -0.6, 0.25 - 0.7j])
    ev = np.linalg.eigvals(st.step_matrix(lam1, 0.0, k))
    for e, l1 in zip(ev, lam1):
        expect = np.array([1.0, l1 ** k, l1 ** k, 0.0])
        assert np.allclose(np.sort_complex(np.round(e, 6)), np.sort_complex(np.round(expect, 6)), atol=1e-5)
    L1, mask = st.zero_stability_region(k, extent=1.5, n=61)
    r = np.abs(L1)
    away = np.abs(r - 1.0) > 0.03
    assert np.array_equal(mask[away], (r < 1.0)[away])


def test_lambda1_zero_gives_the_rk2_region():
    H, mask = st.absolute_stability_region(0.0, k=1, extent=3.0, n=81)
    rk2 = np.abs(1 + H + 0.5 * H * H)
    away = np.abs(rk2 - 1.0) > 1e-3
    assert np.array_equal(mask[away], (rk2 <= 1.0)[away])
    assert mask.any() and not mask.all()


def test_converged_iterations_recover_rk2():
    lam1, lam2 = 0.5 + 0.3j, -0.4 + 0.2j
    h = lam2 / (1 - lam1)
    ev = np.linalg.eigvals(st.step_matrix(lam1, lam2, 200))
    assert np.min(np.abs(ev - (1 + h + 0.5 * h * h))) < 1e-12


@pytest.mark.parametrize("beta_n,beta_p", [(0.0, -4.0), (0.7, -1.0), (-0.3, 2.0)])
def test_constants_are_preserved(beta_n, beta_p):
    A = st.step_matrix(0.3 - 0.4j, 0.0, 3, beta_n=beta_n, beta_p=beta_p)
    one = np.ones(4)
    assert np.abs(A @ one - one).max() < 1e-14


def test_beta_prime_minus_one_is_not_zero_stable_inside_the_disc():
    assert st.spectral_radius(0.7 + 0.25j, 0.0, 1, beta_p=-1.0) > 1.0
    assert st.spectral_radius(0.7 + 0.25j, 0.0, 1, beta_p=-4.0) <= 1.0 + 1e-12
