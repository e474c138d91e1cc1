"""Pins of the oracle's wall-normal bases (App. C) and Fourier transforms
(Section 4, eq. disc_f) against library routines, brute force and closed forms."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle.bspline import SplineSpaces, basis, clamped_knots, derivative_map, greville
from oracle.fourier import n_of_index, to_physical, to_spectral, wavenumbers
from paper_2206_09878_amd.workloads import clustered_breakpoints


def spaces(n2=33, order=8, L2=8.0, gamma=1.5):
    return SplineSpaces(clustered_breakpoints(n2, order, L2, gamma), order)


@pytest.mark.parametrize("order", [4, 8])
def test_basis_matches_scipy(order):
    sp = spaces(n2=25, order=order)
    x = np.linspace(-4.0, 4.0, 157)
    for t, k, n in ((sp.t, order, sp.n2), (sp.ts, order + 1, sp.n2 + 1)):
        B = basis(t, k, x, 2)
        for d in range(3):
            ref = np.stack([BSpline(t, np.eye(n)[j], k - 1)(x, nu=d) for j in range(n)], 1)
            assert np.abs(B[d] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_dimensions_and_greville():
    sp = spaces(n2=33, order=8)
    assert sp.n2 == 33 and sp.ts.size - 9 == 34          # B* has N2+1 functions
    assert sp.tau[0] == -4.0 and abs(sp.tau[-1] - 4.0) < 1e-15
    assert np.all(np.diff(sp.tau) > 0) and np.all(np.diff(sp.tau_s) > 0)
    # clamped ends: B_j(ends) is a Kronecker delta (Dirichlet rows are unit rows)
    assert np.allclose(sp.E[0][0], np.eye(33)[0]) and np.allclose(sp.E[0][-1], np.eye(33)[-1])


def test_partition_of_unity_and_polynomial_reproduction():
    sp = spaces()
    x = np.random.default_rng(0).uniform(-4, 4, 200)
    B = basis(sp.t, sp.order, x, 2)
    assert np.abs(B[0].sum(1) - 1).max() < 1e-14
    # degree <= p-1 polynomials are interpolated exactly at the Greville points
    poly = np.polynomial.Polynomial([0.3, -1.2, 0.5, 0.7, -0.2, 0.05, 0.01, -0.003])
    c = np.linalg.solve(sp.E[0], poly(sp.tau))
    assert np.abs(B[0] @ c - poly(x)).max() < 1e-11
    assert np.abs(B[1] @ c - poly.deriv(1)(x)).max() < 1e-10
    assert np.abs(B[2] @ c - poly.deriv(2)(x)).max() < 1e-9


def test_derivative_map_exact():
    """d/dy of a B* spline lies in the B space with coefficients D* c (App. C)."""
    sp = spaces()
    c = np.random.default_rng(1).standard_normal(sp.n2 + 1)
    ref = BSpline(sp.ts, c, sp.order).derivative()
    assert np.allclose(ref.t, sp.t)
    assert np.abs(ref.c[:sp.n2] - sp.Dstar @ c).max() < 1e-12
    x = np.linspace(-4, 4, 301)
    Bs = basis(sp.ts, sp.order + 1, x, 1)
    B = basis(sp.t, sp.order, x, 0)
    assert np.abs(Bs[1] @ c - B[0] @ (sp.Dstar @ c)).max() < 1e-12
    # kernel of D* is the constants: B* reproduces 1
    assert np.abs(sp.Dstar @ np.ones(sp.n2 + 1)).max() < 1e-12


def test_collocation_matrices_are_banded_and_nonsingular():
    sp = spaces(n2=65)
    for M in (sp.E[0], sp.Es[0]):
        r, c = np.nonzero(M)
        assert max(abs(r - c)) <= 7
        assert np.linalg.cond(M) < 1e3


# ---------------------------------------------------------------------------
# Fourier


def brute_inverse(V, M1, M3):
    ny, nn, nl = V.shape
    n = n_of_index(nn + 1)
    a = np.arange(M1)
    b = np.arange(M3)
    u = np.zeros((ny, M3, M1), dtype=complex)
    for ni in range(nn):
        for l in range(-(nl - 1), nl):
            if l >= 0:
                coef = V[:, ni, l]
                nn_ = n[ni]
            else:
                coef = np.conj(V[:, ni, -l])
                nn_ = -n[ni]
            ph = np.exp(2j * np.pi * (l * a[None, :] / M1 + nn_ * b[:, None] / M3))
            u += coef[:, None, None] * ph[None]
    return u


def rand_hermitian(rng, ny, N1, N3):
    V = rng.standard_normal((ny, N3 - 1, N1 // 2)) + 1j * rng.standard_normal((ny, N3 - 1, N1 // 2))
    nn = N3 - 1
    for ni in range(1, N3 // 2):
        V[:, nn - ni, 0] = np.conj(V[:, ni, 0])
    V[:, 0, 0] = V[:, 0, 0].real
    return V


@pytest.mark.parametrize("N1,N3,M1,M3", [(6, 6, 9, 9), (8, 4, 12, 6), (6, 8, 8, 12)])
def test_transforms_match_brute_force_sums(N1, N3, M1, M3):
    rng = np.random.default_rng(2)
    V = rand_hermitian(rng, 3, N1, N3)
    u = to_physical(V, M1, M3)
    ub = brute_inverse(V, M1, M3)
    assert np.abs(ub.imag).max() < 1e-12
    assert np.abs(u - ub.real).max() < 1e-12
    # forward = (1/(M1 M3)) sum u e^{-i(...)} on the retained modes
    n = n_of_index(N3)
    a, b = np.arange(M1), np.arange(M3)
    Vb = np.zeros_like(V)
    for ni in range(N3 - 1):
        for l in range(N1 // 2):
            ph = np.exp(-2j * np.pi * (l * a[None, :] / M1 + n[ni] * b[:, None] / M3))
            Vb[:, ni, l] = (u * ph[None]).sum((1, 2)) / (M1 * M3)
    assert np.abs(to_spectral(u, N1, N3) - Vb).max() < 1e-13
    assert np.abs(Vb - V).max() < 1e-12            # forward o inverse = identity


def test_parseval():
    rng = np.random.default_rng(3)
    N, M = 16, 24
    V = rand_hermitian(rng, 2, N, N)
    u = to_physical(V, M, M)
    w = np.full(V.shape[1:], 2.0)
    w[:, 0] = 1.0                                   # l = 0 column counted once
    energy = (w[None] * np.abs(V) ** 2).sum((1, 2))
    assert np.allclose((u ** 2).mean((1, 2)), energy, rtol=1e-13)


@pytest.mark.parametrize("N", [8, 16])
def test_three_halves_rule_products_are_exact(N):
    """Products of band-limited fields on the 3N/2 grid give the exact
    (brute-force convolution) coefficients on every retained mode."""
    rng = np.random.default_rng(4)
    M = 3 * N // 2
    A = rand_hermitian(rng, 1, N, N)
    B = rand_hermitian(rng, 1, N, N)
    P = to_spectral(to_physical(A, M, M) * to_physical(B, M, M), N, N)
    # brute force convolution over the full (l, n) plane
    h = N // 2 - 1
    def full(V):
        F = {}
        n = n_of_index(N)
        for ni in range(N - 1):
            for l in range(N // 2):
                F[(l, n[ni])] = V[0, ni, l]
                F[(-l, -n[ni])] = np.conj(V[0, ni, l])
        return F
    FA, FB = full(A), full(B)
    n = n_of_index(N)
    for ni in range(N - 1):
        for l in range(N // 2):
            s = 0
            for (la, na), va in FA.items():
                key = (l - la, n[ni] - na)
                if key in FB:
                    s += va * FB[key]
            assert abs(P[0, ni, l] - s) < 1e-12 * (1 + abs(s))
    # on a grid that is too small the same product aliases
    Ms = N
    Pa = to_spectral(to_physical(A, Ms, Ms) * to_physical(B, Ms, Ms), N, N)
    assert np.abs(Pa - P).max() > 1e-6


def test_derivative_multipliers():
    """i k1, i k3 multipliers are d/dx1, d/dx3 of the physical field."""
    N, M, L1, L3 = 8, 12, 2.0, 3.0
    k1, k3, ksq = wavenumbers(N, N, L1, L3)
    V = np.zeros((1, N - 1, N // 2), complex)
    V[0, 2, 3] = 0.3 - 0.2j                         # l = 3, n = 2
    x = np.arange(M) * L1 / M
    z = np.arange(M) * L3 / M
    ph = 3 * 2 * np.pi * x[None, :] / L1 + 2 * 2 * np.pi * z[:, None] / L3
    c = 0.3 - 0.2j
    exact = 2 * (c * np.exp(1j * ph)).real
    assert np.abs(to_physical(V, M, M)[0] - exact).max() < 1e-14
    d1 = to_physical(1j * k1[None, None, :] * V, M, M)[0]
    d3 = to_physical(1j * k3[None, :, None] * V, M, M)[0]
    assert np.abs(d1 - 2 * (1j * 3 * 2 * np.pi / L1 * c * np.exp(1j * ph)).real).max() < 1e-13
    assert np.abs(d3 - 2 * (1j * 2 * 2 * np.pi / L3 * c * np.exp(1j * ph)).real).max() < 1e-13
    assert ksq[2, 3] == pytest.approx((3 * 2 * np.pi / L1) ** 2 + (2 * 2 * np.pi / L3) ** 2)
