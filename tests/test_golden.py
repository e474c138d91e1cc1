"""Pins against numbers the paper prints (fixtures under tests/golden/, each
with its citation)."""
import json
import math
import os

import numpy as np
import pytest

import oracle.ode_model as om
from oracle.lmvd import bdf_coefficients
from paper_2206_09878_amd.workloads import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_model_problem_constants_match_the_paper():
    g = load("ode_model.json")
    for k, v in (("c1", om.C1), ("c2", om.C2), ("c3", om.C3), ("c4", om.C4)):
        assert v == complex(*g[k]), k
    # defaults of the oracle's model integration are the paper's
    import inspect
    sig = inspect.signature(om.integrate)
    assert sig.parameters["z0"].default == g["z0"] and sig.parameters["md0"].default == g["md0"]
    assert sig.parameters["beta_p"].default == g["beta_p"] and sig.parameters["beta_n"].default == g["beta_n"]
    assert sig.parameters["kf"].default == g["kf"]


def test_rt512_parameters_match_the_paper_table():
    """The benchmark workload is the At = 0.925, 3D, Re = 1024 case of the table,
    nondimensionalised with rho_h = W = g = 1 (mu = 1/Re)."""
    row = [r for r in load("rt_cases.json")["rows_3d"] if r["At"] == 0.925][0]
    w = workload("rt512")
    at = (w.rho_h - w.rho_l) / (w.rho_h + w.rho_l)
    assert at == pytest.approx(row["At"], rel=1e-12)
    assert w.mu == pytest.approx(1.0 / row["Re"], rel=1e-15)
    assert w.dt * math.sqrt(at) / math.sqrt(w.L1 / w.g) == pytest.approx(row["dt_scaled"], rel=1e-12)


@pytest.mark.parametrize("stage", [0, 1])
def test_guess_coefficients_for_the_printed_betas(stage):
    """With the printed beta values the BDF-like guesses (eq. dzdt_guesses) give
    dz/dt exactly for a history linear in t: the constant moment vanishes and
    the first moment is one.  Stage history offsets (units of dt, most recent
    first): -1/2, -1, -3/2 for both stages (App. A)."""
    g = load("ode_model.json")
    a = np.asarray(bdf_coefficients(stage, g["beta_n"], g["beta_p"]))
    offsets = np.array([0.0, -0.5, -1.0, -1.5])
    assert abs(a.sum()) < 1e-14
    assert abs(a @ offsets - 1.0) < 1e-14
