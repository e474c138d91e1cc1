"""lmvd_substep_noalloc (the substep on the library's own fixed device workspace, for callers that cannot
allocate) against lmvd_substep on a caller workspace, through the C ABI: two calls in a row, the second
on a smaller grid, each bit-identical to the plain entry point.  The plain entry point's workspace is
filled with NaN first, so a substep that read a workspace byte it had not written would show it.  A plan
whose workspace exceeds the fixed array is refused before anything runs."""
import ctypes

import numpy as np
import pytest

from paper_2206_09878_amd.workloads import make_inputs, workload

pytestmark = pytest.mark.gpu


def _run(p, w, inp, noalloc):
    import torch
    from paper_2206_09878_amd.lmvd import _check, _ptr, library
    st = {k: p.to_dev(inp[k]) for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    hist = [p.to_dev(h) for h in inp["hist"]]
    z_out, zt = p.empty(), p.empty()
    rhs = {"phi2": p.empty(), "omega2": p.empty(),
           "m1bar": torch.empty(w.n2, dtype=torch.float64, device="cuda"),
           "m3bar": torch.empty(w.n2, dtype=torch.float64, device="cuda")}
    a = p.substep_args(0, st["phi2"], st["omega2"], st["z"], st["m1bar"], st["m3bar"], z_out=z_out, hist=hist,
                       rhs_out=rhs, zt_out=zt)
    lib = library()
    if noalloc:
        _check(lib.lmvd_substep_noalloc(p.handle, ctypes.byref(a), p._stream()), "lmvd_substep_noalloc")
    else:
        p.ws.view(torch.float64).fill_(float("nan"))
        _check(lib.lmvd_substep(p.handle, ctypes.byref(a), _ptr(p.ws), p._stream()), "lmvd_substep")
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in st.items()}
    out.update(z_out=z_out.cpu().numpy(), zt=zt.cpu().numpy(), **{"rhs_" + k: v.cpu().numpy() for k, v in rhs.items()})
    return out


def test_noalloc_substep_equals_the_plain_entry_point():
    import torch
    from paper_2206_09878_amd.lmvd import Plan, library
    assert torch.cuda.is_available()
    cap = ctypes.c_size_t()
    assert library().lmvd_noalloc_capacity(ctypes.byref(cap)) == 0 and cap.value == 64 << 20
    for n, n2 in ((32, 33), (16, 17)):          # the second call on a smaller grid
        w = workload("small", n=n, n2=n2)
        p = Plan(w)
        assert p.workspace_bytes <= cap.value
        inp = make_inputs(w, seed=21 + n)
        print(f"noalloc substep {n}x{n2}x{n}, workspace {p.workspace_bytes} bytes", flush=True)
        got = _run(p, w, inp, noalloc=True)
        ref = _run(p, w, inp, noalloc=False)
        for k in ref:
            assert np.isfinite(ref[k]).all(), k
            assert np.array_equal(got[k], ref[k]), k


def test_noalloc_refuses_a_workspace_beyond_its_array():
    import torch
    from paper_2206_09878_amd.lmvd import Plan, library
    assert torch.cuda.is_available()
    w = workload("small", n=64, n2=65)
    p = Plan(w)
    assert p.workspace_bytes > 64 << 20
    inp = make_inputs(w, seed=3)
    st = {k: p.to_dev(inp[k]) for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
    z_out = p.empty()
    before = z_out.clone()
    a = p.substep_args(0, st["phi2"], st["omega2"], st["z"], st["m1bar"], st["m3bar"], z_out=z_out,
                       hist=[p.to_dev(h) for h in inp["hist"]], rhs_out={"phi2": p.empty(), "omega2": p.empty(),
                       "m1bar": torch.empty(w.n2, dtype=torch.float64, device="cuda"),
                       "m3bar": torch.empty(w.n2, dtype=torch.float64, device="cuda")}, zt_out=p.empty())
    assert library().lmvd_substep_noalloc(p.handle, ctypes.byref(a), p._stream()) == -4
    torch.cuda.synchronize()
    assert torch.equal(z_out.view(torch.float64).nan_to_num(), before.view(torch.float64).nan_to_num())
