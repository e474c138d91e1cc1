"""CPU checks of the C ABI: the library loads, exports every declared entry
point, validates configurations, and its host plan builder (own B-spline
code) agrees with the oracle's spline spaces."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2206_09878_amd import lmvd
from paper_2206_09878_amd.workloads import workload
from oracle.bspline import SplineSpaces

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lmvd.h")).read()
    return sorted(set(re.findall(r"\b(lmvd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lmvd.library()
    syms = declared_symbols()
    assert "lmvd_substep" in syms and len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) <= set(lmvd.EXPORTS)


def test_status_strings():
    lib = lmvd.library()
    assert lib.lmvd_status_string(0) == b"ok"
    assert b"invalid" in lib.lmvd_status_string(-1)
    assert b"non-finite" in lib.lmvd_status_string(-6)


def test_config_layout_matches_the_header(tmp_path):
    """The ctypes mirror of lmvd_config has the C struct's size and field offsets (gcc, host only)."""
    import subprocess
    fields = [f[0] for f in lmvd.Config._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lmvd.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(lmvd_config));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(lmvd_config, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(lmvd.Config)
    assert got[1:] == [getattr(lmvd.Config, f).offset for f in fields]


@pytest.mark.parametrize("change", ["rhoD_form", "check_finite", "mu_z_nan", "rhoD_z_inf"])
def test_plan_create_rejects_bad_transport_laws_and_flags(change):
    cfg = lmvd.make_config(workload("small"))
    if change == "rhoD_form":
        cfg.rhoD_form = 2
    elif change == "check_finite":
        cfg.check_finite = 3
    elif change == "mu_z_nan":
        cfg.mu_z[1] = float("nan")
    else:
        cfg.rhoD_z[0] = float("inf")
    h = ctypes.c_void_p()
    assert lmvd.library().lmvd_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == -1


@pytest.mark.parametrize("name,n,n2", [("small", None, None), ("small", 16, 25), ("mixing128", 48, 65)])
def test_host_tables_match_oracle(name, n, n2):
    w = workload(name, n=n, n2=n2)
    tau, taus, E = lmvd.host_tables(w)
    sp = SplineSpaces(w.breakpoints, w.order)
    assert np.abs(tau - sp.tau).max() < 1e-14 * w.L2
    assert np.abs(taus - sp.tau_s).max() < 1e-14 * w.L2
    for d in range(3):
        scale = np.abs(sp.E[d]).max()
        assert np.abs(E[d] - sp.E[d]).max() < 1e-12 * scale, d


@pytest.mark.parametrize("field,value,status", [
    ("n1", 31, -1),          # odd
    ("m1", 20, -1),          # m1 < n1
    ("order", 12, -4),       # unsupported order
    ("dt", -1.0, -1),
    ("m3", 5 * 48, None),    # m3 not 2^a 3^b -> unsupported
])
def test_plan_create_rejects_bad_configs(field, value, status):
    w = workload("small")
    cfg = lmvd.make_config(w)
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    st = lmvd.library().lmvd_plan_create(ctypes.byref(cfg), ctypes.byref(h))
    assert st != 0
    if status is not None:
        assert st == status


def test_bad_breakpoints_rejected():
    w = workload("small")
    cfg = lmvd.make_config(w)
    bp = np.array(w.breakpoints)
    bp[3], bp[4] = bp[4], bp[3]
    cfg.breakpoints = bp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert lmvd.library().lmvd_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == -1


@pytest.mark.parametrize("n1,n3,n2,order", [(32, 32, 4097, 8), (32, 1024, 33, 8)])
def test_plan_create_rejects_sizes_beyond_the_kernels(n1, n3, n2, order):
    """n2 above 4096 (plane-mean kernel LDS) and M3 above 1024 (z transforms): LMVD_EUNSUPPORTED from
    the host checks, before any allocation."""
    import dataclasses
    w = dataclasses.replace(workload("small"), n1=n1, n3=n3, n2=n2, m1=3 * n1 // 2, m3=3 * n3 // 2, order=order)
    cfg = lmvd.make_config(w)
    h = ctypes.c_void_p()
    assert lmvd.library().lmvd_plan_create(ctypes.byref(cfg), ctypes.byref(h)) == -4


@pytest.mark.parametrize("name", ["small", "mixing128", "rt512"])
def test_factor_check_host_passes_on_the_workload_grids(name):
    """Every distinct k of the grid (27,239 at 512x385x512 with its clustered knots) passes the pivot
    check of the A(k) elimination; the growth stays near 1 and the pivots far from zero."""
    from paper_2206_09878_amd.lmvd import factor_check_host
    w = workload(name)
    st, growth, pivot, bad, nk = factor_check_host(w)
    assert st == 0 and bad == 0
    assert nk > (w.n1 // 2) * (w.n3 // 2) // 4
    assert 1.0 <= growth < 2.0 and pivot > 1e-2


def test_factor_check_host_fires_below_the_growth_it_sees():
    """A growth limit below the growth the elimination reaches makes rows fail (LMVD_ENUMERIC): the check
    is live."""
    from paper_2206_09878_amd.lmvd import factor_check_host
    w = workload("small")
    st, growth, _, _, _ = factor_check_host(w)
    assert st == 0
    st, _, _, bad, _ = factor_check_host(w, growth_max=0.5 * (1.0 + growth))
    assert st == -5 and bad > 0


@pytest.mark.parametrize("struct,cname", [("SubstepGrads", "lmvd_substep_grads"), ("SubstepArgs", "lmvd_substep_args")])
def test_argument_struct_layouts_match_the_header(tmp_path, struct, cname):
    """The ctypes mirrors of lmvd_substep_grads and lmvd_substep_args have the C structs' size and field
    offsets (gcc, host only)."""
    import subprocess
    cls = getattr(lmvd, struct)
    fields = [f[0] for f in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lmvd.h"\nint main(void) {\n'
                   f'  printf("%zu\\n", sizeof({cname}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({cname}, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, f).offset for f in fields]


def test_basis_values_match_scipy():
    """lmvd_basis_values (the plan builder's Cox-de Boor at arbitrary y) against scipy's B-splines on the
    same knots, for B (order p) and B* (order p + 1), including both walls."""
    from scipy.interpolate import BSpline
    from paper_2206_09878_amd.lmvd import basis_values
    w = workload("small", n=16, n2=25)
    sp = SplineSpaces(w.breakpoints, w.order)
    y = np.concatenate([[-w.L2 / 2, w.L2 / 2], np.random.default_rng(3).uniform(-w.L2 / 2, w.L2 / 2, 40)])
    for star, t, k in ((False, sp.t, w.order - 1), (True, sp.ts, w.order)):
        got = basis_values(w, y, star=star)
        ref = BSpline.design_matrix(np.clip(y, t[0], t[-1] - 1e-15 * w.L2), t, k).toarray()
        ref[1] = 0.0
        ref[1, -1] = 1.0                           # the right end: the last basis function alone
        assert np.abs(got - ref).max() < 1e-12, star
    with pytest.raises(lmvd.LmvdError):
        basis_values(w, [w.L2])
