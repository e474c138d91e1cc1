"""The z-tile autotuner (lmvd_autotune) through the C ABI:

  * every tile divisor D = 1, 2, 4 gives the oracle's substep at 1e-11, and
    the same bits as the other divisors (each z line is transformed by the same
    threads in the same order; only the number of lines per block changes);
  * the timed choice is one of the candidates, with a time for each;
  * plans without a tile choice (768-point z lines, sizes without a register
    plan) keep D = 1;
  * a graph of tuned instances of uneven sizes equals their eager substeps;
  * the graph-level tuner (timing the graph itself) leaves the results unchanged.
"""
import pytest

from paper_2206_09878_amd.workloads import batch_workloads, make_inputs, workload
from tests.test_gpu_parity import check_pair, host, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.mark.parametrize("n,n2", [(32, 33), (48, 49), (64, 65)])
def test_every_tile_matches_the_oracle_and_each_other(torch, n, n2):
    w = workload("small", n=n, n2=n2)
    outs = {}
    for d in (1, 2, 4):
        print("tile", d, (n, n2, n), flush=True)
        got, ref = run_pair(w, 0, seed=50, tile=d)
        check_pair(got, ref)
        outs[d] = got
    for d in (2, 4):
        for k in ("phi2", "omega2", "z", "zt"):
            assert (outs[d][k] == outs[1][k]).all(), (d, k)


def test_timed_choice(torch):
    from paper_2206_09878_amd.lmvd import Plan
    p = Plan(workload("small", n=32, n2=33))
    d, t = p.autotune()
    print("choice", d, "times (ms)", t, flush=True)
    assert d in (1, 2, 4)
    assert all(x > 0 for x in t)
    assert t[(1, 2, 4).index(d)] == min(t)


def test_no_choice_without_register_z_kernels(torch):
    from paper_2206_09878_amd.lmvd import Plan
    for w in (workload("small", n=24, n2=25), workload("rt512", n=512, n2=9)):   # M3 = 36, 768
        d, t = Plan(w).autotune()
        assert d == 1 and t == [-1.0, -1.0, -1.0]


def test_graph_of_tuned_instances(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    ws = batch_workloads(count=5, seed=4000)
    mk = lambda: [Stepper(Plan(w), make_inputs(w, seed=w.extra["seed"], stage=0), stage=0) for w in ws]
    A, B = mk(), mk()
    for i, s in enumerate(A):
        s.p.autotune(force=(1, 2, 4)[i % 3])
    g = GraphBatch(A, nsub=4)
    for _ in range(2):
        for s in B:
            for _ in range(4):
                s.substep()
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip(A, B):
            for k in ("z", "phi2", "omega2", "m1bar", "m3bar"):
                assert torch.equal(a.state()[k], b.state()[k]), k


def test_graph_autotune_keeps_the_results(torch):
    """lmvd_graph_autotune times the graph itself (its tries advance the
    instances); afterwards the recaptured graph still equals eager substeps
    started from the same state, bit for bit."""
    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    ws = batch_workloads(count=6, seed=4100)
    mk = lambda: [Stepper(Plan(w), make_inputs(w, seed=w.extra["seed"], stage=0), stage=0) for w in ws]
    A, B = mk(), mk()
    g = GraphBatch(A, nsub=4)
    tiles, ms = g.autotune(launches=1)
    print("graph tiles", tiles, "ms per launch", ms, flush=True)
    assert len(tiles) == 6 and all(t in (1, 2, 4) for t in tiles) and ms > 0
    for a, b in zip(A, B):
        sa, sb = a.state(), b.state()
        assert sa["stage"] == sb["stage"] == 0
        for k in ("z", "phi2", "omega2", "m1bar", "m3bar", "zt", "zt_next"):
            sb[k].copy_(sa[k])
        for x, y in zip(sa["hist"], sb["hist"]):
            y.copy_(x)
        for k in sa["rhs"]:
            sb["rhs"][k].copy_(sa["rhs"][k])
    torch.cuda.synchronize()
    for _ in range(2):
        for s in B:
            for _ in range(4):
                s.substep()
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip(A, B):
            for k in ("z", "phi2", "omega2", "m1bar", "m3bar"):
                assert torch.equal(a.state()[k], b.state()[k]), k
