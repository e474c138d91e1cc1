"""The non-finite check of lmvd_substep (check_finite in lmvd_config):
finite substeps pass, a NaN in the state is reported as LMVD_ENONFINITE after
the substep has run, a plan without the flag runs on silently, and a plan
with it cannot enter a graph (the check synchronises the stream)."""
import pytest

from paper_2206_09878_amd.workloads import make_inputs, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def stepper(check):
    from paper_2206_09878_amd.lmvd import Plan, Stepper
    w = workload("small", n=16, n2=25)
    return Stepper(Plan(w, check_finite=check), make_inputs(w, seed=40, stage=0), stage=0)


def test_finite_substeps_pass_and_nan_is_reported(torch):
    from paper_2206_09878_amd.lmvd import LmvdError
    s = stepper(True)
    for _ in range(2):
        s.substep()
    torch.cuda.synchronize()
    s.z[3, 2, 1] = complex(float("nan"), 0.0)
    with pytest.raises(LmvdError, match="non-finite"):
        s.substep()
    assert not torch.isfinite(torch.view_as_real(s.z)).all()


def test_without_the_flag_nan_passes_silently(torch):
    s = stepper(False)
    s.substep()
    s.z[3, 2, 1] = complex(float("nan"), 0.0)
    s.substep()
    torch.cuda.synchronize()
    assert not torch.isfinite(torch.view_as_real(s.z)).all()


def test_a_checked_plan_cannot_enter_a_graph(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch, LmvdError
    with pytest.raises(LmvdError):
        GraphBatch([stepper(True)], nsub=4)
