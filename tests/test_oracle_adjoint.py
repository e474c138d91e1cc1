"""Pins of the transposes used by the library's adjoint operators, on the
oracle's own (separately pinned) transforms and spline matrices:

  * the inverse transform's transpose in the real inner products is
    M1 M3 w_l times the forward transform, w_0 = 1, w_l = 2 (l > 0), for any
    spectral array, Hermitian l = 0 column or not;
  * a direct check of that identity against the transform written as a dense
    real matrix on a tiny grid (brute force)."""
import numpy as np

from oracle.fourier import to_physical, to_spectral


def rdot(a, b):
    return float(np.sum((np.conj(a) * b).real))


def transform_transpose(g, N1, N3):
    M3, M1 = g.shape[1], g.shape[2]
    d = to_spectral(g, N1, N3) * (M1 * M3)
    d[:, :, 1:] *= 2.0
    return d


def test_inverse_transform_transpose_identity():
    rng = np.random.default_rng(3)
    for (N1, N3, M1, M3) in ((8, 8, 12, 12), (16, 12, 24, 18), (32, 32, 48, 48)):
        shape = (3, N3 - 1, N1 // 2)
        c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        g = rng.standard_normal((3, M3, M1))
        lhs = float(np.sum(to_physical(c, M1, M3) * g))
        rhs = rdot(c, transform_transpose(g, N1, N3))
        assert abs(lhs - rhs) < 1e-12 * np.abs(c).sum() * np.abs(g).max()


def test_transpose_against_a_dense_real_matrix():
    """Tiny grid: build the real matrix of c -> to_physical(c) column by column
    (real and imaginary unit inputs) and compare its transpose with the formula."""
    N1, N3, M1, M3 = 6, 6, 9, 9
    shape = (1, N3 - 1, N1 // 2)
    n = int(np.prod(shape))
    cols = []
    for k in range(2 * n):
        e = np.zeros(2 * n)
        e[k] = 1.0
        c = (e[:n] + 1j * e[n:]).reshape(shape)
        cols.append(to_physical(c, M1, M3).ravel())
    A = np.array(cols).T                                   # physical <- (Re c, Im c)
    rng = np.random.default_rng(5)
    g = rng.standard_normal((1, M3, M1))
    d = transform_transpose(g, N1, N3).ravel()
    At_g = A.T @ g.ravel()
    assert np.abs(At_g - np.concatenate([d.real, d.imag])).max() < 1e-12
