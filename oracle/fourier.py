"""Fourier representation in the two homogeneous directions (Section 4, eq. disc_f).

Test infrastructure only: nothing in the product path imports this module.

A field is the truncated series sum_{l,n} f_ln(y) exp(i k1 x1) exp(i k3 x3) with
l in [-(N1/2-1), N1/2-1], n in [-(N3/2-1), N3/2-1] (the Nyquist modes are
excluded), k1 = 2 pi l / L1, k3 = 2 pi n / L3.  The field is real, so
f_{-l,-n} = conj(f_{l,n}) and only l >= 0 is stored.

Storage layout of a spectral array (oracle and library alike): shape
[ny, N3-1, N1/2], index [j, n_idx, l]; n_idx runs over n = 0 .. N3/2-1 and then
n = -(N3/2-1) .. -1.

The paper does not describe dealiasing.  Reading used here: nonlinear products
are formed on an M1 x M3 physical grid (3/2 rule, M = 3N/2), x_a = a L1/M1,
z_b = b L3/M3; the inverse transform is the plain (unnormalised) sum over the
retained modes and the forward transform is (1/(M1 M3)) sum_{a,b} u e^{-i(...)},
kept on the retained modes only.  A library FFT (numpy) evaluates both sums.
"""
from __future__ import annotations

import numpy as np


def n_of_index(N3: int) -> np.ndarray:
    """Wavenumber index n for each stored n_idx."""
    h = N3 // 2
    return np.concatenate([np.arange(0, h), np.arange(-(h - 1), 0)])


def wavenumbers(N1, N3, L1, L3):
    """k1[l], k3[n_idx] and k^2 as a [N3-1, N1/2] array."""
    l = np.arange(N1 // 2)
    n = n_of_index(N3)
    k1 = 2.0 * np.pi * l / L1
    k3 = 2.0 * np.pi * n / L3
    ksq = k3[:, None] ** 2 + k1[None, :] ** 2
    return k1, k3, ksq


def to_physical(V: np.ndarray, M1: int, M3: int) -> np.ndarray:
    """Inverse transform: values V[j, n_idx, l] -> real field u[j, b, a].

    u(x_a, z_b) = sum over retained (l, n) of V_ln e^{i(k1 x_a + k3 z_b)}, with
    the l < 0 half supplied by V_{-l,-n} = conj(V_{l,n}).  For l = 0 both n
    and -n are stored; the real part of the sum is returned, which is the
    real field of the Hermitian part of the l = 0 column.
    """
    ny, nn, nl = V.shape
    N3 = nn + 1
    n = n_of_index(N3)
    full = np.zeros((ny, M3, M1), dtype=np.complex128)
    for ni in range(nn):
        full[:, n[ni] % M3, 0:nl] = V[:, ni, :]
        # negative l half from the Hermitian partner of (l, n)
        full[:, (-n[ni]) % M3, (M1 - np.arange(1, nl)) % M1] = np.conj(V[:, ni, 1:])
    u = np.fft.ifft2(full, axes=(1, 2)) * (M1 * M3)
    return u.real.copy()


def to_spectral(u: np.ndarray, N1: int, N3: int) -> np.ndarray:
    """Forward transform: real field u[j, b, a] -> values V[j, n_idx, l]."""
    ny, M3, M1 = u.shape
    S = np.fft.fft2(u, axes=(1, 2)) / (M1 * M3)
    n = n_of_index(N3)
    V = np.empty((ny, N3 - 1, N1 // 2), dtype=np.complex128)
    for ni in range(N3 - 1):
        V[:, ni, :] = S[:, n[ni] % M3, 0:N1 // 2]
    return V
