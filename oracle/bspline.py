"""Wall-normal B-spline bases of the oracle (Appendix C, "Spatial discretization").

Test infrastructure only: nothing in the product path imports this module.

The paper represents every field except the wall-normal momentum m2 with
maximum-continuity B-splines B_j of order p on a set of breakpoints, and m2
with B-splines B*_j of order p+1 on the same breakpoints, so that dB*_j/dy
spans the space of the B_j (App. C, eq. disc_f_inhomo and the paragraph after
it; subsection "B-splines").  The order, the knot placement and the
collocation points are not given for the results; the readings used here are

* clamped (open) knot vectors: each end breakpoint repeated `order` times,
  interior breakpoints once (maximum continuity);
* collocation points = Greville abscissae of the knot vector.

Basis values are computed from the Cox-de Boor recursion and derivatives from
the standard derivative recursion (de Boor, "A Practical Guide to Splines"),
written out directly.  Everything is float64.
"""
from __future__ import annotations

import numpy as np


def clamped_knots(breakpoints: np.ndarray, order: int) -> np.ndarray:
    """Clamped knot vector of a maximum-continuity spline space of `order`.

    With nb breakpoints the space has nb + order - 2 functions.
    """
    xi = np.asarray(breakpoints, dtype=np.float64)
    if xi.ndim != 1 or xi.size < 2 or np.any(np.diff(xi) <= 0):
        raise ValueError("breakpoints must be strictly increasing")
    return np.concatenate([np.full(order - 1, xi[0]), xi, np.full(order - 1, xi[-1])])


def greville(knots: np.ndarray, order: int) -> np.ndarray:
    """Greville abscissae: tau_i = mean(t_{i+1}, ..., t_{i+order-1})."""
    n = knots.size - order
    return np.array([knots[i + 1:i + order].mean() for i in range(n)])


def basis(knots: np.ndarray, order: int, x, nderiv: int = 0) -> np.ndarray:
    """All B-splines of `order` on `knots` and their derivatives at points x.

    Returns B with B[d, q, j] = d^d B_j / dy^d at x[q], for d = 0..nderiv.
    The right end of the knot vector belongs to the last nonempty interval.
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nt = t.size
    # Order-1 splines: indicator of [t_j, t_{j+1}); the last nonempty
    # interval is closed on the right.
    last = np.nonzero(t[1:] > t[:-1])[0][-1]
    ind = np.zeros((x.size, nt - 1))
    for j in range(nt - 1):
        if t[j + 1] > t[j]:
            if j == last:
                ind[:, j] = (x >= t[j]) & (x <= t[j + 1])
            else:
                ind[:, j] = (x >= t[j]) & (x < t[j + 1])
    # table[k][d] holds d-th derivatives of all order-k splines (nt - k of them)
    table = {1: {0: ind}}
    for d in range(1, nderiv + 1):
        table[1][d] = np.zeros_like(ind)

    def ratio(num, den):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)

    for k in range(2, order + 1):
        n = nt - k
        j = np.arange(n)
        left_den = t[j + k - 1] - t[j]          # t_{j+k-1} - t_j
        right_den = t[j + k] - t[j + 1]         # t_{j+k} - t_{j+1}
        prev = table[k - 1]
        cur = {}
        # Cox-de Boor: B_{j,k} = w_left B_{j,k-1} + w_right B_{j+1,k-1}
        wl = ratio(x[:, None] - t[j][None, :], left_den[None, :])
        wr = ratio(t[j + k][None, :] - x[:, None], right_den[None, :])
        cur[0] = wl * prev[0][:, :n] + wr * prev[0][:, 1:n + 1]
        # derivative: D B_{j,k} = (k-1)[B_{j,k-1}/left_den - B_{j+1,k-1}/right_den]
        for d in range(1, nderiv + 1):
            cur[d] = (k - 1) * (ratio(prev[d - 1][:, :n], left_den[None, :])
                                - ratio(prev[d - 1][:, 1:n + 1], right_den[None, :]))
        table[k] = cur
    return np.stack([table[order][d] for d in range(nderiv + 1)])


def derivative_map(knots_star: np.ndarray, order_star: int) -> np.ndarray:
    """Coefficient map D* of the derivative of an order-`order_star` spline.

    If s = sum_j c_j B*_j (order p+1 on knots t*), then ds/dy = sum_j d_j B_j
    with B_j of order p on t*[1:-1] and
        d_j = p (c_{j+1} - c_j) / (t*_{j+p+1} - t*_{j+1}).
    Returns the (n-1) x n matrix D* (App. C: dB*/dy spans the B space).
    """
    t = np.asarray(knots_star, dtype=np.float64)
    k = order_star
    n = t.size - k
    D = np.zeros((n - 1, n))
    for j in range(n - 1):
        w = (k - 1) / (t[j + k] - t[j + 1])
        D[j, j] = -w
        D[j, j + 1] = w
    return D


class SplineSpaces:
    """The B (order p) and B* (order p+1) spaces on one set of breakpoints.

    Attributes (n2 = number of B functions):
      t, ts        knot vectors of B and B*
      tau          Greville points of B (n2 points, both ends included):
                   the physical y-grid
      tau_s        Greville points of B* (n2+1 points)
      E[d]         E_d[i, j]  = d^d B_j  (tau_i),   d = 0, 1, 2
      Es[d]        E*_d[i, j] = d^d B*_j (tau*_i),  d = 0, 1, 2
      F[d]         F_d[i, j]  = d^d B*_j (tau_i),   d = 0, 1
      G[d]         G_d[i, j]  = d^d B_j  (tau*_i),  d = 0, 1
      Dstar        B-coefficients of d/dy of a B* spline
    """

    def __init__(self, breakpoints, order: int = 8):
        self.order = order
        self.breakpoints = np.asarray(breakpoints, dtype=np.float64)
        self.t = clamped_knots(self.breakpoints, order)
        self.ts = clamped_knots(self.breakpoints, order + 1)
        self.n2 = self.t.size - order
        self.tau = greville(self.t, order)
        self.tau_s = greville(self.ts, order + 1)
        self.E = basis(self.t, order, self.tau, 2)
        self.Es = basis(self.ts, order + 1, self.tau_s, 2)
        self.F = basis(self.ts, order + 1, self.tau, 1)
        self.G = basis(self.t, order, self.tau_s, 1)
        self.Dstar = derivative_map(self.ts, order + 1)
