"""Seeded synthetic workloads: problem sizes, physical parameters and input fields.

This module only synthesises inputs.  It contains none of the method's
arithmetic (no transforms, products, spline evaluations or solves): every
field is produced directly as arrays of spectral B-spline coefficients from
random numbers and closed-form profiles, so the same inputs can be handed to
the HIP library and to an independent checker.

Workloads (shapes and parameters of the paper's Rayleigh-Taylor runs,
Section 5 and Appendix D, and of a mixing layer):

  small        32 x 33 x 32 Fourier/B-spline modes, 48 x 48 physical x-z grid,
               density ratio 3, broadband k^-5/3 momentum (k <= 8)
  mixing128    128 x 129 x 128 (192 x 192), density 1 -> 7 across a tanh layer
               of width 0.05 L2, 1 % broadband perturbation
  rt512        512 x 385 x 512 (768 x 768), At = 0.925 (density ratio 25.67),
               Re = 1024, g = 1, interface perturbed by modes 4..64
  adjoint96    96 x 97 x 96 (144 x 144), density ratio 7 layer
  batch        (batch_workloads) 64 small instances of uneven sizes, N1, N3 in
               {32, 48, 64, 96}, n2 in {33, 49, 65, 97}, density ratio 2..25

Array layout (all spectral arrays): complex128 [ny, N3-1, N1/2], index
[j, n_idx, l], with n_idx covering n = 0..N3/2-1 then n = -(N3/2-1)..-1.
The l = 0 column is Hermitian in n (f_{0,-n} = conj f_{0,n}); (0,0) is real.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def clustered_breakpoints(n2: int, order: int, L2: float, gamma: float) -> np.ndarray:
    """n2 - order + 2 breakpoints on [-L2/2, L2/2] clustered at y = 0:
    y(s) = (L2/2) artanh(s tanh(gamma)) / gamma, s uniform in [-1, 1]."""
    nb = n2 - order + 2
    s = np.linspace(-1.0, 1.0, nb)
    y = 0.5 * L2 * np.arctanh(s * np.tanh(gamma)) / gamma
    y[0], y[-1] = -0.5 * L2, 0.5 * L2
    return y


def sample_points(n2: int, L2: float, gamma: float) -> np.ndarray:
    """n2 points through the same clustering map; used only to shape the
    synthetic coefficient profiles."""
    s = np.linspace(-1.0, 1.0, n2)
    y = 0.5 * L2 * np.arctanh(s * np.tanh(gamma)) / gamma
    y[0], y[-1] = -0.5 * L2, 0.5 * L2
    return y


@dataclass
class Workload:
    name: str
    n1: int
    n3: int
    n2: int
    m1: int
    m3: int
    L1: float
    L2: float
    L3: float
    gamma: float
    dt: float
    mu: float
    rhoD: float
    g: float
    rho_l: float
    rho_h: float
    order: int = 8
    kf: int = 4
    beta_n: float = 0.0
    beta_p: float = -4.0
    extra: dict = field(default_factory=dict)
    # transport laws (Section 2): mu(z) = mu + sum_k mu_z[k] z^(k+1);
    # rho D_z = q(z) (rhoD_form 0) or f(z) q(z) (1), q(z) = rhoD + sum_k rhoD_z[k] z^(k+1)
    mu_z: tuple = (0.0, 0.0, 0.0)
    rhoD_z: tuple = (0.0, 0.0, 0.0)
    rhoD_form: int = 0

    @property
    def breakpoints(self) -> np.ndarray:
        return clustered_breakpoints(self.n2, self.order, self.L2, self.gamma)

    @property
    def shape(self):
        return (self.n2, self.n3 - 1, self.n1 // 2)

    @property
    def shape_star(self):
        return (self.n2 + 1, self.n3 - 1, self.n1 // 2)


def workload(name: str, n: int | None = None, n2: int | None = None) -> Workload:
    """The named workload; `n`, `n2` override the grid (M = 3n/2)."""
    if name == "small":
        w = Workload("small", 32, 32, 33, 48, 48, 2 * math.pi, 8.0, 2 * math.pi, 1.5,
                     dt=1e-3, mu=1e-2, rhoD=1e-2, g=0.0, rho_l=1.0, rho_h=3.0,
                     extra=dict(delta=0.5, kmax=8, amp=0.1, zpert=0.02, env=2.0))
    elif name == "mixing128":
        w = Workload("mixing128", 128, 128, 129, 192, 192, 2 * math.pi, 2 * math.pi,
                     2 * math.pi, 1.5, dt=2e-3, mu=1e-3, rhoD=1e-3, g=0.0,
                     rho_l=1.0, rho_h=7.0,
                     extra=dict(delta=0.05 * 2 * math.pi, kmax=42, amp=0.01, zpert=0.01,
                                env=4 * 0.05 * 2 * math.pi))
    elif name == "rt512":
        at = 0.925
        rho_h = 1.0
        rho_l = rho_h * (1 - at) / (1 + at)
        w = Workload("rt512", 512, 512, 385, 768, 768, 1.0, 7.0, 1.0, 2.0,
                     dt=3.125e-5 / math.sqrt(at), mu=1.0 / 1024, rhoD=1.0 / 1024, g=1.0,
                     rho_l=rho_l, rho_h=rho_h,
                     extra=dict(eps=0.05, h0=0.5, kmin=4, kmax=64, hrms=0.01))
    elif name == "adjoint96":
        w = Workload("adjoint96", 96, 96, 97, 144, 144, 2 * math.pi, 2 * math.pi,
                     2 * math.pi, 1.5, dt=2e-3, mu=1e-3, rhoD=1e-3, g=0.0,
                     rho_l=1.0, rho_h=7.0,
                     extra=dict(delta=0.05 * 2 * math.pi, kmax=32, amp=0.01, zpert=0.01,
                                env=4 * 0.05 * 2 * math.pi))
    else:
        raise KeyError(name)
    if n is not None:
        w.n1 = w.n3 = n
        w.m1 = w.m3 = 3 * n // 2
        w.extra = dict(w.extra)
        if "kmax" in w.extra:
            w.extra["kmax"] = min(w.extra["kmax"], n // 2 - 1)
    if n2 is not None:
        w.n2 = n2
    return w


def batch_workloads(count: int = 64, seed: int = 1000) -> list:
    """`count` independent small instances of uneven sizes (the batched mode):
    instance i draws, from default_rng(seed + i), N1 and N3 from {32, 48, 64, 96},
    n2 from {33, 49, 65, 97} and a density ratio rho_h / rho_l from U[2, 25];
    everything else as `small` (its inputs come from make_inputs(w, seed + i))."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n1 = int(rng.choice([32, 48, 64, 96]))
        n3 = int(rng.choice([32, 48, 64, 96]))
        n2 = int(rng.choice([33, 49, 65, 97]))
        ratio = float(rng.uniform(2.0, 25.0))
        w = workload("small")
        w.name = f"batch{i}"
        w.n1, w.n3, w.n2 = n1, n3, n2
        w.m1, w.m3 = 3 * n1 // 2, 3 * n3 // 2
        w.rho_l, w.rho_h = 1.0, ratio
        w.extra = dict(w.extra, means="jet", kmax=min(w.extra["kmax"], min(n1, n3) // 2 - 1), seed=seed + i)
        out.append(w)
    return out


# ----------------------------------------------------------------------------


def _mode_grid(w: Workload):
    h = w.n3 // 2
    n = np.concatenate([np.arange(0, h), np.arange(-(h - 1), 0)])
    l = np.arange(w.n1 // 2)
    kap = np.sqrt(n[:, None] ** 2 + l[None, :] ** 2)
    return n, l, kap


def _hermitian_l0(a: np.ndarray) -> np.ndarray:
    """Make the l = 0 column Hermitian in n and the (0,0) entry real."""
    nn = a.shape[1]
    h = (nn + 1) // 2
    for ni in range(1, h):
        a[:, nn - ni, 0] = np.conj(a[:, ni, 0])
    a[:, 0, 0] = a[:, 0, 0].real
    return a


def _random_modes(rng, w: Workload, amp_of_kappa, profile):
    """a(kappa) * profile(y_j) * complex normal, Hermitian on l = 0."""
    n, l, kap = _mode_grid(w)
    a = amp_of_kappa(kap)
    xi = (rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)) / math.sqrt(2)
    f = xi * a[None] * profile[:, None, None]
    return _hermitian_l0(f)


def broadband_momentum(w: Workload, seed: int, amp: float = 1e-3, kmax: int = 32):
    """(phi2, Omega2) coefficient arrays with k^-5/3 amplitudes for 1 <= kappa <= kmax, a Gaussian
    profile across the channel (zero at the walls) and random complex normal entries: a broadband m^d to
    add to states that have none (the Rayleigh-Taylor initial state), so that every product of the
    substep is non-trivial."""
    rng = np.random.default_rng(seed)
    n, l, kap = _mode_grid(w)
    a = np.where((kap >= 1) & (kap <= kmax), np.maximum(kap, 1.0) ** (-5.0 / 3.0), 0.0)
    prof = np.exp(-np.linspace(-2.0, 2.0, w.n2) ** 2)
    prof[0] = prof[-1] = 0.0

    def field():
        xi = rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)
        return _hermitian_l0(amp * xi * a[None] * prof[:, None, None])
    return field(), field()


def make_inputs(w: Workload, seed: int = 0, stage: int = 0) -> dict:
    """Seeded inputs of one substep.

    Returns dict of numpy arrays:
      phi2, omega2, z          complex [n2, N3-1, N1/2] B coefficients
      m1bar, m3bar             float [n2]
      hist                     list of 3 z coefficient arrays, previous
                               stages most recent first, from a smooth
                               synthetic dz/dt (z - dt/2 zdot, z - dt zdot,
                               z - 3/2 dt zdot for stage n; z - dt/2 zdot,
                               z - dt zdot, z - 3/2 dt zdot relative to the
                               stage-n value for stage ')
      rhs_prev, zt_prev        (stage ' only) smooth stage-n RHS data
    """
    rng = np.random.default_rng(seed)
    y = sample_points(w.n2, w.L2, w.gamma)
    ex = w.extra
    n, l, kap = _mode_grid(w)
    shape = w.shape
    z = np.zeros(shape, dtype=np.complex128)
    phi2 = np.zeros(shape, dtype=np.complex128)
    omega2 = np.zeros(shape, dtype=np.complex128)
    m1bar = np.zeros(w.n2)
    m3bar = np.zeros(w.n2)
    if w.name == "rt512":
        W = w.L1
        width = 2 * ex["eps"] * W
        z[:, 0, 0] = 0.5 * (1.0 + np.tanh((y - ex["h0"] * W) / width))
        # interface h(x, z) = h0 + sum_{kmin <= |k| <= kmax} a cos(k.x + phase),
        # linearised: z_ln(y) = -h_ln dz0/dy
        mask = (kap >= ex["kmin"]) & (kap <= ex["kmax"])
        ph = rng.uniform(0, 2 * math.pi, size=kap.shape)
        hln = np.where(mask, np.exp(1j * ph), 0.0)
        hln[:, 0] = 0.0       # keep l > 0 modes; the l = 0 column is filled
        nl0 = (n > 0) & (np.abs(n) >= ex["kmin"]) & (np.abs(n) <= ex["kmax"])
        hln[nl0, 0] = np.exp(1j * ph[nl0, 0])
        # rms of a real field with these half-spectrum modes: sqrt(2 sum |h|^2)
        hln *= ex["hrms"] * W / math.sqrt(2.0 * np.sum(np.abs(hln) ** 2))
        dz0 = 0.5 / width / np.cosh((y - ex["h0"] * W) / width) ** 2
        z += -hln[None] * dz0[:, None, None]
        z = _hermitian_l0(z)
    else:
        delta = ex["delta"]
        z[:, 0, 0] = 0.5 * (1.0 + np.tanh(y / delta))
        env = np.exp(-(y / ex["env"]) ** 2)
        env[0] = env[-1] = 0.0
        amp = lambda k: np.where((k >= 1) & (k <= ex["kmax"]), np.maximum(k, 1.0) ** (-5.0 / 3.0), 0.0)
        # phi2 ~ k^2 m2: scale so that velocities are O(amp)
        kk = 2 * math.pi / w.L1
        phi2 = ex["amp"] * (kk ** 2) * _random_modes(rng, w, lambda k: amp(k) * np.maximum(k, 1.0) ** 2, env)
        omega2 = ex["amp"] * kk * _random_modes(rng, w, lambda k: amp(k) * np.maximum(k, 1.0), env)
        zenv = np.exp(-(y / (2 * delta)) ** 2)
        z += ex["zpert"] * _random_modes(rng, w, amp, zenv)
        z[:, 0, 0] = 0.5 * (1.0 + np.tanh(y / delta))
        if ex.get("means", "jet" if w.name == "small" else "shear") == "shear":
            # mean shear across the layer: <m>1 ~ rho_mean(y) * dU/2 tanh(y/delta)
            rho_mean = w.rho_l + (w.rho_h - w.rho_l) * 0.5 * (1 + np.tanh(y / delta))
            m1bar = rho_mean * 0.5 * np.tanh(y / delta)
        else:
            m1bar = 0.05 * np.exp(-(y / ex["env"]) ** 2)
            m3bar = -0.03 * np.exp(-(y / ex["env"]) ** 2) * y / ex["env"]
    # smooth synthetic time derivative of z for the history
    zdot_env = np.exp(-(y / (0.25 * w.L2)) ** 2)
    zdot = 0.05 * _random_modes(rng, w, lambda k: np.where(k <= 6, 1.0 / (1.0 + k) ** 2, 0.0), zdot_env)
    dt = w.dt
    out = dict(phi2=phi2, omega2=omega2, z=z, m1bar=m1bar, m3bar=m3bar)
    if stage == 0:
        out["hist"] = [z - 0.5 * dt * zdot, z - dt * zdot, z - 1.5 * dt * zdot]
    else:
        # stage ': current z is z' = z^n + dt/2 zdot
        zn = z - 0.5 * dt * zdot
        out["hist"] = [zn, zn - 0.5 * dt * zdot, zn - dt * zdot]
        prof = np.exp(-(y / (0.25 * w.L2)) ** 2)
        prof_d = prof.copy()
        prof_d[0] = prof_d[-1] = 0.0
        sm = lambda k: np.where(k <= 6, 1.0 / (1.0 + k) ** 2, 0.0)
        out["rhs_prev"] = dict(
            phi2=_random_modes(rng, w, sm, prof_d),
            omega2=_random_modes(rng, w, sm, prof_d),
            m1bar=0.1 * prof, m3bar=-0.05 * prof)
        out["rhs_prev"]["phi2"][:, 0, 0] = 0
        out["rhs_prev"]["omega2"][:, 0, 0] = 0
        out["zt_prev"] = zdot.copy()
    return out
