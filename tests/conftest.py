"""Shared fixtures.  Tests marked `gpu` need an MI355X and the built HIP library."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def oracle_config(w):
    """Oracle Config of a workload (test helper)."""
    from oracle.lmvd import Config
    return Config(w.n1, w.n3, w.n2, w.order, w.m1, w.m3, w.L1, w.L2, w.L3,
                  w.breakpoints, w.dt, w.mu, w.rhoD, w.g, w.rho_l, w.rho_h,
                  w.beta_n, w.beta_p, w.kf, tuple(w.mu_z), tuple(w.rhoD_z), w.rhoD_form)
