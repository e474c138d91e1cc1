"""Linear stability of the time discretisation (Section 3.3.2, Appendix B):
amplification matrices and stability regions of the scheme on the model
problem dz/dt = lambda1 dz/dt + lambda2 z.

Per stage the scheme guesses dz/dt from the z history (eq. dzdt_guesses),
applies k fixed-point iterations zt <- lambda1 zt + lambda2 z, and advances z
with explicit midpoint RK2.  On the history vector
x = [z^n, z^{n-1,'}, z^{n-1}, z^{n-2,'}] one step is x -> A2 A1 x with

  A1 (stage n):  z' = z^n + dt/2 zt^n,             x' = [z', z^n, z^{n-1,'}, z^{n-1}]
  A2 (stage '):  z^{n+1} = z^n + dt zt',           x'' = [z^{n+1}, z', z^n, z^{n-1,'}]

(z^{n+1} = z' + dt (zt' - zt^n / 2) and zt^n = 2 (z' - z^n) / dt), where after
k iterations dt zt = Lambda g + S z, Lambda = lambda1^k, S = dt lambda2
(1 + lambda1 + ... + lambda1^{k-1}), g the stage's guess times dt.  The lower
three rows of both matrices shift the history; the first row is the stage's
physical update.  (Written out here from the scheme; the matrices printed in
the paper's appendix do not preserve constants and are not used.)

Zero stability (lambda2 = 0): with beta^n = 0, beta' = -4 the eigenvalues are
{1, lambda1^k, lambda1^k, 0}, so the scheme is zero-stable exactly when
|lambda1| < 1, for every k.  Fully converged (k -> infinity) the physical
eigenvalue is the RK2 polynomial of h = dt lambda2 / (1 - lambda1).

    python -m paper_2206_09878_amd.stability [--k 2] [--beta-p -4] [--lam1 0.5+0.3j] [--extent 3] [--n 61]

prints the absolute-stability region in the dt lambda2 plane for one
lambda1, and the zero-stability region in the lambda1 plane.
"""
from __future__ import annotations

import argparse

import numpy as np


def guess_weights(stage: int, beta_n: float = 0.0, beta_p: float = -4.0) -> np.ndarray:
    """Weights of eq. dzdt_guesses on [z^s, previous three stage values] (most recent first)."""
    if stage == 0:
        return np.array([2.0, -(2.0 + 0.5 * beta_n), beta_n, -0.5 * beta_n])
    return np.array([4.0 + beta_p, -(5.0 + 2.0 * beta_p), beta_p, 1.0])


def _iteration_factors(lam1, lam2dt, k: int):
    """Lambda = lambda1^k and S = dt lambda2 sum_{j<k} lambda1^j (broadcast arrays)."""
    lam1 = np.asarray(lam1, dtype=complex)
    lam2dt = np.asarray(lam2dt, dtype=complex)
    geo = np.zeros(np.broadcast(lam1, lam2dt).shape, dtype=complex)
    p = np.ones_like(geo)
    for _ in range(k):
        geo = geo + p
        p = p * lam1
    return p, lam2dt * geo


def stage_matrices(lam1, lam2dt, k: int, beta_n: float = 0.0, beta_p: float = -4.0):
    """(A1, A2), each [..., 4, 4], broadcast over lam1 and lam2dt."""
    Lam, S = _iteration_factors(lam1, lam2dt, k)
    shape = Lam.shape
    I4 = np.eye(4)
    A1 = np.zeros(shape + (4, 4), dtype=complex)
    A2 = np.zeros(shape + (4, 4), dtype=complex)
    a = guess_weights(0, beta_n, beta_p)
    b = guess_weights(1, beta_n, beta_p)
    # stage n: dt zt^n = Lambda a.x + S z^n;  z' = z^n + dt zt^n / 2
    A1[..., 0, :] = I4[0] + 0.5 * (Lam[..., None] * a + S[..., None] * I4[0])
    # stage ': dt zt' = Lambda b.x' + S z';  z^{n+1} = z^n + dt zt'  (z^n is x'[1])
    A2[..., 0, :] = Lam[..., None] * b + S[..., None] * I4[0] + I4[1]
    for A in (A1, A2):
        A[..., 1, 0] = 1.0
        A[..., 2, 1] = 1.0
        A[..., 3, 2] = 1.0
    return A1, A2


def step_matrix(lam1, lam2dt, k: int, beta_n: float = 0.0, beta_p: float = -4.0) -> np.ndarray:
    A1, A2 = stage_matrices(lam1, lam2dt, k, beta_n, beta_p)
    return A2 @ A1


def spectral_radius(lam1, lam2dt, k: int, beta_n: float = 0.0, beta_p: float = -4.0) -> np.ndarray:
    return np.abs(np.linalg.eigvals(step_matrix(lam1, lam2dt, k, beta_n, beta_p))).max(axis=-1)


def absolute_stability_region(lam1: complex, k: int, extent: float = 3.0, n: int = 61,
                              beta_n: float = 0.0, beta_p: float = -4.0, tol: float = 1e-9):
    """Grid of h = dt lambda2 in [-extent, extent]^2 and the mask rho(A) <= 1 + tol."""
    x = np.linspace(-extent, extent, n)
    H = x[None, :] + 1j * x[::-1, None]
    return H, spectral_radius(lam1, H, k, beta_n, beta_p) <= 1.0 + tol


def zero_stability_region(k: int, extent: float = 1.5, n: int = 61, beta_n: float = 0.0,
                          beta_p: float = -4.0, tol: float = 1e-9):
    """Grid of lambda1 in [-extent, extent]^2 and the mask rho(A(lambda1, 0)) <= 1 + tol."""
    x = np.linspace(-extent, extent, n)
    L1 = x[None, :] + 1j * x[::-1, None]
    return L1, spectral_radius(L1, 0.0, k, beta_n, beta_p) <= 1.0 + tol


def _ascii(mask: np.ndarray) -> str:
    return "\n".join("".join("#" if v else "." for v in row) for row in mask)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--beta-n", type=float, default=0.0)
    ap.add_argument("--beta-p", type=float, default=-4.0)
    ap.add_argument("--lam1", type=complex, default=0.5 + 0.3j)
    ap.add_argument("--extent", type=float, default=3.0)
    ap.add_argument("--n", type=int, default=61)
    a = ap.parse_args()
    H, m = absolute_stability_region(a.lam1, a.k, a.extent, a.n, a.beta_n, a.beta_p)
    print(f"absolute stability, lambda1 = {a.lam1}, k = {a.k}, beta' = {a.beta_p}: dt lambda2 in "
          f"[-{a.extent}, {a.extent}]^2 (# stable), area {m.mean() * (2 * a.extent) ** 2:.3f}")
    print(_ascii(m))
    L1, z = zero_stability_region(a.k, 1.5, a.n, a.beta_n, a.beta_p)
    print(f"zero stability, k = {a.k}: lambda1 in [-1.5, 1.5]^2")
    print(_ascii(z))


if __name__ == "__main__":
    main()
