"""Independent simulations of uneven sizes in one HIP graph (lmvd_graph_*),
through the C ABI.

  * Every graph launch equals the same substeps run one by one on the plain
    path, bit for bit (same kernels, same inputs, no atomics), over several
    launches with eager work and synchronisations between them.
  * Uneven instances (N1 != N3, n2 = 49 and 97) match the oracle within 1e-11
    on one substep, so the graph's results inherit the parity of the plain path.
  * Instances whose substeps do not line up (different k_f) take the
    one-branch-per-instance form of the graph, with the same bit-for-bit result.
  * The entry point rejects diagnostic outputs and a period that breaks the
    history ring.
  * Instances at row counts 14, 19 and 22 (other tails of the unrolled column
    sweeps) are bit for bit equal to their eager substeps as well.
"""
import ctypes

import numpy as np
import pytest

from paper_2206_09878_amd.workloads import batch_workloads, make_inputs
from tests.test_gpu_parity import TOL, check_pair, host, rel, rhs_tolerances, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def steppers(ws):
    from paper_2206_09878_amd.lmvd import Plan, Stepper
    return [Stepper(Plan(w), make_inputs(w, seed=w.extra["seed"], stage=0), stage=0) for w in ws]


def state_tensors(s):
    st = s.state()
    out = [st["z"], *st["hist"], st["phi2"], st["omega2"], st["m1bar"], st["m3bar"], st["zt"], st["zt_next"]]
    out += [st["rhs"][k] for k in sorted(st["rhs"])]
    return out


def test_graph_replays_equal_eager_substeps(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch
    ws = batch_workloads(count=6)
    print("graph instances:", [(w.n1, w.n2, w.n3) for w in ws], flush=True)
    A, B = steppers(ws), steppers(ws)
    g = GraphBatch(A, nsub=4)
    assert g.grouped
    for launch in range(3):
        for s in B:
            for _ in range(4):
                s.substep()
        g.launch()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(A, B)):
            assert a.stage == b.stage == 0
            for ta, tb in zip(state_tensors(a), state_tensors(b)):
                assert ta.data_ptr() != tb.data_ptr()
                assert torch.equal(ta, tb), (launch, i)
        # the state keeps moving: the next launch starts from a new state
        assert np.isfinite(host(A[0].z)).all()


def test_graph_row_counts(torch):
    """Instances whose row counts (n2 = 14, 19, 22) end the unrolled column sweeps in other tails than
    the batch's n2 = 2^k + 1, grouped in one graph, equal the same substeps run one by one, bit for bit."""
    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    from paper_2206_09878_amd.workloads import workload
    ws = [workload("small", n=16, n2=n2) for n2 in (14, 19, 22)]

    def make():
        return [Stepper(Plan(w), make_inputs(w, seed=60 + w.n2, stage=0), stage=0) for w in ws]

    A, B = make(), make()
    g = GraphBatch(A, nsub=4)
    print("row-count instances:", [(w.n1, w.n2, w.n3) for w in ws], "grouped", g.grouped, flush=True)
    for launch in range(2):
        for s in B:
            for _ in range(4):
                s.substep()
        g.launch()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(A, B)):
            for ta, tb in zip(state_tensors(a), state_tensors(b)):
                assert torch.equal(ta, tb), (launch, i)


def test_graph_eight_substeps_per_launch(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch
    ws = batch_workloads(count=3, seed=2000)
    A, B = steppers(ws), steppers(ws)
    g = GraphBatch(A, nsub=8)
    g.launch()
    for s in B:
        for _ in range(8):
            s.substep()
    torch.cuda.synchronize()
    for a, b in zip(A, B):
        for ta, tb in zip(state_tensors(a), state_tensors(b)):
            assert torch.equal(ta, tb)


def test_graph_mixed_iteration_counts_fall_back_to_branches(torch):
    """Instances whose substeps differ step by step (k_f = 4, 2, 4) cannot share
    grouped launches; the graph then runs one branch per instance.  Still equal
    to the plain path, bit for bit, over two launches."""
    from paper_2206_09878_amd.lmvd import GraphBatch
    ws = batch_workloads(count=3, seed=3000)
    kfs = [4, 2, 4]
    A, B = steppers(ws), steppers(ws)
    g = GraphBatch(A, nsub=4, kf=kfs)
    assert not g.grouped
    for launch in range(2):
        for s, kf in zip(B, kfs):
            for _ in range(4):
                s.substep(kf=kf)
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip(A, B):
            for ta, tb in zip(state_tensors(a), state_tensors(b)):
                assert torch.equal(ta, tb), launch


@pytest.mark.parametrize("pick", ["n2_49", "n2_97"])
def test_uneven_instance_matches_oracle(torch, pick):
    ws = batch_workloads(count=64)
    n2 = int(pick.split("_")[1])
    w = next(x for x in ws if x.n1 != x.n3 and x.n2 == n2)
    print("instance", w.name, (w.n1, w.n2, w.n3), "ratio", round(w.rho_h, 3), flush=True)
    got, ref = run_pair(w, 0, seed=w.extra["seed"])
    check_pair(got, ref, rhs_tol=rhs_tolerances(w, 0, w.extra["seed"], ref=ref))


def test_graph_rejects_bad_arguments(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch, LmvdError, SubstepArgs, library
    ws = batch_workloads(count=1)
    (s,) = steppers(ws)
    with pytest.raises(LmvdError):
        GraphBatch([s], nsub=3)
    # diagnostic outputs are not allowed in a graph
    a = s.next_args()
    a.md[0] = s.z.data_ptr()
    arr = (SubstepArgs * 1)(a)
    plans = (ctypes.c_void_p * 1)(s.p.handle.value)
    wsp = (ctypes.c_void_p * 1)(s.p.ws.data_ptr())
    h = ctypes.c_void_p()
    assert library().lmvd_graph_create(plans, arr, wsp, 1, 1, ctypes.byref(h)) != 0
    assert library().lmvd_graph_create(plans, arr, wsp, 0, 1, ctypes.byref(h)) != 0


def test_substeps_captured_in_a_caller_graph(torch):
    """lmvd_substep allocates, memsets and synchronises nothing, so a caller can capture it: four
    substeps captured with torch.cuda.graph, replayed three times with eager work and synchronisations
    in between, equal the same substeps run eagerly, bit for bit, after every replay."""
    ws = batch_workloads(count=1, seed=5000)
    (a,), (b,) = steppers(ws), steppers(ws)
    a.substep()
    b.substep()
    for _ in range(3):               # back to the start of the history-ring period
        a.substep()
        b.substep()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(4):
                a.substep()
    torch.cuda.synchronize()
    for replay in range(3):
        g.replay()
        for _ in range(4):
            b.substep()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work between replays
        for ta, tb in zip(state_tensors(a), state_tensors(b)):
            assert torch.equal(ta, tb), replay
        assert torch.isfinite(junk)


@pytest.mark.parametrize("split", [3, 4])
def test_checkpoint_resume_is_bit_identical(torch, tmp_path, split):
    """Stepper.save after `split` substeps (stage ' or n next), Stepper.load on a fresh plan, then the
    remaining substeps: the same bits as the uninterrupted run."""
    from paper_2206_09878_amd.lmvd import Plan, Stepper
    (w,) = batch_workloads(count=1, seed=5100)
    (a,) = steppers([w])
    for _ in range(split):
        a.substep()
    path = str(tmp_path / "state.npz")
    a.save(path)
    b = Stepper.load(Plan(w), path)
    assert b.stage == a.stage
    for _ in range(8 - split):
        a.substep()
        b.substep()
    torch.cuda.synchronize()
    for k in ("z", "phi2", "omega2", "m1bar", "m3bar"):
        assert torch.equal(a.state()[k], b.state()[k]), k
