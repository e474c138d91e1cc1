"""The z-tile autotuner (lmvd_autotune) through the C ABI:

  * every tile code K = D + 8 V (line plan V: threads per line, radix split and stage order; divisor D of
    the lines per block) gives the oracle's substep at the five register z sizes (M3 = 48, 72, 96, 144,
    192), each output within 1e-11 or 4 x the oracle's own FFT-rounding spread where that is larger
    (the stage RHS at 128 x 17 x 128, whose k^2-weighted mean-shear flux amplifies rounding); codes of one
    plan give the same bits (each z line is transformed by the same threads in the same order; only the
    number of lines per block changes), and the plans agree with each other within the same bounds;
  * the timed choice is one of the candidates, with a time for each;
  * plans without a tile choice (768-point z lines, sizes without a register plan) keep K = 1;
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


@pytest.mark.parametrize("n,n2", [(32, 33), (48, 49), (64, 65), (96, 33), (128, 17)])
def test_every_tile_matches_the_oracle_and_each_other(torch, n, n2):
    from tests.test_gpu_parity import gpu_substep, oracle_substep, output_errors, spread_tolerances
    w = workload("small", n=n, n2=n2)
    inp = make_inputs(w, seed=50, stage=0)
    ref = oracle_substep(w, 0, inp)
    tol = spread_tolerances(w, 0, ref, inp)
    nplans = 3 if w.m3 in (48, 72, 96, 144, 192) else 1
    codes = [d + 8 * v for v in range(nplans) for d in (1, 2, 4)]
    outs = {}
    for k in codes:
        print("tile", k, (n, n2, n), flush=True)
        got = gpu_substep(w, 0, inp, tile=k)
        check_pair(got, ref, tols=tol)
        outs[k] = got
    for k in codes:
        base = outs[k - (k % 8) + 1]                 # the same plan with D = 1
        for key in ("phi2", "omega2", "z", "zt"):
            assert (outs[k][key] == base[key]).all(), (k, key)
        other = {"state": outs[1], "zt": outs[1]["zt"], "rhs": outs[1]["rhs"],
                 "diag": {"md": outs[1]["md"], "mc": outs[1]["mc"]}}
        errs = output_errors(outs[k], other)
        bad = {key: (v, tol[key]) for key, v in errs.items() if not v < tol[key]}
        assert not bad, (k, bad)


def test_timed_choice(torch):
    from paper_2206_09878_amd.lmvd import Plan
    p = Plan(workload("small", n=32, n2=33))
    d, t = p.autotune()
    print("choice", d, "times (ms)", t, flush=True)
    assert d in p.TILE_CODES
    assert all(x > 0 for x in t)                     # M3 = 48: three plans, every code timed
    assert t[p.TILE_CODES.index(d)] == min(t)


def test_no_choice_without_register_z_kernels(torch):
    from paper_2206_09878_amd.lmvd import Plan
    for w in (workload("small", n=24, n2=25), workload("rt512", n=512, n2=9)):   # M3 = 36, 768
        d, t = Plan(w).autotune()
        assert d == 1 and t == [-1.0] * 9


def test_graph_of_tuned_instances(torch):
    from paper_2206_09878_amd.lmvd import GraphBatch, Plan, Stepper
    ws = batch_workloads(count=5, seed=4000)
    mk = lambda: [Stepper(Plan(w), make_inputs(w, seed=w.extra["seed"], stage=0), stage=0) for w in ws]
    A, B = mk(), mk()
    # the eager twins run the same line plans (plans differ from each other in rounding)
    for i, (a, b) in enumerate(zip(A, B)):
        k = (1, 2, 4, 9, 12, 18, 20)[i % 7]
        a.p.autotune(force=k)
        b.p.autotune(force=k - k % 8 + 1)
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
    assert len(tiles) == 6 and all(t in Plan.TILE_CODES for t in tiles) and ms > 0
    for t, b in zip(tiles, B):
        b.p.autotune(force=t - t % 8 + 1)     # the same line plan, divisor 1
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
