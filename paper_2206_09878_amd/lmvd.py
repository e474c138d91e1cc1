"""Python binding of the HIP library (ctypes; argument marshalling only).

Every step of the substep runs in the library's kernels; torch supplies device
memory and the current stream.  The binding loads the in-tree
``_lmvd.so`` and raises if it is missing: there is no CPU fallback.

Spectral arrays are torch.complex128 tensors of shape [ny, N3-1, N1/2]
(index [j, n_idx, l]) on the GPU; plane means are float64 [n2].
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lmvd.so")
_lib = None


class LmvdError(RuntimeError):
    pass


class Config(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n3", ctypes.c_int32), ("n2", ctypes.c_int32), ("order", ctypes.c_int32),
        ("m1", ctypes.c_int32), ("m3", ctypes.c_int32),
        ("L1", ctypes.c_double), ("L2", ctypes.c_double), ("L3", ctypes.c_double),
        ("breakpoints", ctypes.POINTER(ctypes.c_double)),
        ("dt", ctypes.c_double), ("mu", ctypes.c_double), ("rhoD", ctypes.c_double), ("g", ctypes.c_double),
        ("rho_l", ctypes.c_double), ("rho_h", ctypes.c_double),
        ("beta_n", ctypes.c_double), ("beta_p", ctypes.c_double),
        ("kf", ctypes.c_int32), ("plane_batch", ctypes.c_int32),
        ("mu_z", ctypes.c_double * 3), ("rhoD_z", ctypes.c_double * 3), ("rhoD_form", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
    ]


class SubstepArgs(ctypes.Structure):
    _fields_ = [
        ("stage", ctypes.c_int32), ("kf", ctypes.c_int32), ("guess_mode", ctypes.c_int32),
        ("phi2", ctypes.c_void_p), ("omega2", ctypes.c_void_p), ("z", ctypes.c_void_p),
        ("m1bar", ctypes.c_void_p), ("m3bar", ctypes.c_void_p),
        ("phi2_out", ctypes.c_void_p), ("omega2_out", ctypes.c_void_p), ("z_out", ctypes.c_void_p),
        ("m1bar_out", ctypes.c_void_p), ("m3bar_out", ctypes.c_void_p),
        ("rhs_phi2_prev", ctypes.c_void_p), ("rhs_omega2_prev", ctypes.c_void_p), ("zt_prev", ctypes.c_void_p),
        ("rhs_m1_prev", ctypes.c_void_p), ("rhs_m3_prev", ctypes.c_void_p),
        ("rhs_phi2", ctypes.c_void_p), ("rhs_omega2", ctypes.c_void_p), ("zt", ctypes.c_void_p),
        ("rhs_m1", ctypes.c_void_p), ("rhs_m3", ctypes.c_void_p),
        ("z_hist", ctypes.c_void_p * 3),
        ("md", ctypes.c_void_p * 3), ("mc", ctypes.c_void_p * 3),
    ]


_V = ctypes.c_void_p


class SubstepGrads(ctypes.Structure):
    """Mirror of lmvd_substep_grads: output cotangents, then input gradients."""
    _fields_ = ([(n, _V) for n in ("phi2_out", "omega2_out", "z_out", "m1bar_out", "m3bar_out", "rhs_phi2",
                                   "rhs_omega2", "zt", "rhs_m1", "rhs_m3")]
                + [("md", _V * 3), ("mc", _V * 3)]
                + [(n, _V) for n in ("phi2", "omega2", "z", "m1bar", "m3bar")]
                + [("z_hist", _V * 3)]
                + [(n, _V) for n in ("rhs_phi2_prev", "rhs_omega2_prev", "zt_prev", "rhs_m1_prev", "rhs_m3_prev")])


EXPORTS = ["lmvd_status_string", "lmvd_plan_create", "lmvd_plan_destroy", "lmvd_sizes", "lmvd_substep",
           "lmvd_to_physical", "lmvd_to_spectral", "lmvd_project", "lmvd_evaluate", "lmvd_md", "lmvd_mc",
           "lmvd_host_tables", "lmvd_profile_start", "lmvd_profile_stop", "lmvd_graph_create",
           "lmvd_graph_launch", "lmvd_graph_destroy", "lmvd_graph_grouped", "lmvd_autotune",
           "lmvd_graph_autotune", "lmvd_rhs", "lmvd_to_physical_adjoint", "lmvd_evaluate_adjoint",
           "lmvd_project_adjoint", "lmvd_md_adjoint", "lmvd_mc_adjoint", "lmvd_to_spectral_adjoint",
           "lmvd_factor_check", "lmvd_factor_check_host", "lmvd_substep_noalloc", "lmvd_noalloc_capacity",
           "lmvd_adjoint_sizes", "lmvd_substep_adjoint", "lmvd_basis_values"]


def library():
    """Load the built library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise LmvdError(f"HIP library not built: {_LIB_PATH} (run python -m paper_2206_09878_amd.build)")
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.lmvd_status_string.restype = ctypes.c_char_p
        lib.lmvd_status_string.argtypes = [ctypes.c_int]
        lib.lmvd_plan_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
        lib.lmvd_plan_destroy.argtypes = [vp]
        lib.lmvd_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t)]
        lib.lmvd_substep.argtypes = [vp, ctypes.POINTER(SubstepArgs), vp, vp]
        lib.lmvd_substep_noalloc.argtypes = [vp, ctypes.POINTER(SubstepArgs), vp]
        lib.lmvd_noalloc_capacity.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        lib.lmvd_adjoint_sizes.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
        lib.lmvd_basis_values.argtypes = [ctypes.POINTER(Config), i32, vp, i32, vp]
        lib.lmvd_substep_adjoint.argtypes = [vp, ctypes.POINTER(SubstepArgs), ctypes.POINTER(SubstepGrads), vp, vp]
        lib.lmvd_to_physical.argtypes = [vp, vp, vp, vp, vp]
        lib.lmvd_to_spectral.argtypes = [vp, vp, vp, vp, vp]
        lib.lmvd_project.argtypes = [vp, i32, vp, vp, vp]
        lib.lmvd_evaluate.argtypes = [vp, i32, i32, vp, vp, vp]
        lib.lmvd_md.argtypes = [vp] * 8 + [vp, vp]
        lib.lmvd_mc.argtypes = [vp] * 7
        lib.lmvd_rhs.argtypes = [vp] * 11
        lib.lmvd_to_physical_adjoint.argtypes = [vp] * 5
        lib.lmvd_evaluate_adjoint.argtypes = [vp, i32, i32, vp, vp, vp]
        lib.lmvd_project_adjoint.argtypes = [vp, i32, vp, vp, vp]
        lib.lmvd_md_adjoint.argtypes = [vp] * 10
        lib.lmvd_mc_adjoint.argtypes = [vp] * 7
        lib.lmvd_to_spectral_adjoint.argtypes = [vp] * 5
        lib.lmvd_host_tables.argtypes = [ctypes.POINTER(Config), vp, vp, vp, vp, vp]
        pd, p64 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        lib.lmvd_factor_check.argtypes = [vp, ctypes.c_double, pd, pd, p64]
        lib.lmvd_factor_check_host.argtypes = [ctypes.POINTER(Config), ctypes.c_double, pd, pd, p64, p64]
        lib.lmvd_profile_start.argtypes = [vp, i32, i32]
        lib.lmvd_profile_stop.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_double)]
        lib.lmvd_graph_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SubstepArgs), ctypes.POINTER(vp), i32,
                                          i32, ctypes.POINTER(vp)]
        lib.lmvd_graph_launch.argtypes = [vp, vp]
        lib.lmvd_graph_destroy.argtypes = [vp]
        lib.lmvd_graph_grouped.argtypes = [vp, ctypes.POINTER(i32)]
        lib.lmvd_autotune.argtypes = [vp, vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        lib.lmvd_graph_autotune.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SubstepArgs), ctypes.POINTER(vp), i32,
                                            i32, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        for name in EXPORTS:
            if name != "lmvd_status_string":
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(st: int, what: str):
    if st != 0:
        msg = library().lmvd_status_string(st).decode()
        raise LmvdError(f"{what}: {msg} ({st})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_config(w, plane_batch: int = 0, check_finite: bool = False):
    """ctypes Config from a workload (paper_2206_09878_amd.workloads.Workload).
    The returned object keeps its breakpoint buffer alive."""
    bp = np.ascontiguousarray(w.breakpoints, dtype=np.float64)
    c = Config(w.n1, w.n3, w.n2, w.order, w.m1, w.m3, w.L1, w.L2, w.L3,
               bp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), w.dt, w.mu, w.rhoD, w.g,
               w.rho_l, w.rho_h, w.beta_n, w.beta_p, w.kf, plane_batch,
               (ctypes.c_double * 3)(*w.mu_z), (ctypes.c_double * 3)(*w.rhoD_z), w.rhoD_form, int(check_finite))
    c._bp = bp
    return c


def host_tables(w):
    """Greville points and E_d matrices of the plan builder (host only)."""
    cfg = make_config(w)
    n2 = w.n2
    tau = np.zeros(n2)
    taus = np.zeros(n2 + 1)
    E = [np.zeros((n2, n2)) for _ in range(3)]
    st = library().lmvd_host_tables(ctypes.byref(cfg), tau.ctypes.data, taus.ctypes.data,
                                    E[0].ctypes.data, E[1].ctypes.data, E[2].ctypes.data)
    _check(st, "lmvd_host_tables")
    return tau, taus, E


def basis_values(w, y, star: bool = False):
    """Values of the B (B* with star) basis at the points y (host): array [len(y), n2 (+1)]."""
    cfg = make_config(w)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros((len(y), w.n2 + (1 if star else 0)))
    _check(library().lmvd_basis_values(ctypes.byref(cfg), len(y), y.ctypes.data, int(star), out.ctypes.data),
           "lmvd_basis_values")
    return out


def factor_check_host(w, growth_max: float = 1e4):
    """Pivot check of the A(k) elimination for every distinct k of the workload's grid, on the host
    (lmvd_factor_check_host).  Returns (status, max growth, min pivot ratio, failed rows, distinct k)."""
    cfg = make_config(w)
    g, r = ctypes.c_double(), ctypes.c_double()
    bad, nk = ctypes.c_int64(), ctypes.c_int64()
    st = library().lmvd_factor_check_host(ctypes.byref(cfg), growth_max, ctypes.byref(g), ctypes.byref(r),
                                          ctypes.byref(bad), ctypes.byref(nk))
    if st not in (0, -5):
        _check(st, "lmvd_factor_check_host")
    return st, g.value, r.value, bad.value, nk.value


class Plan:
    """A plan plus its workspace on the current GPU."""

    def __init__(self, w, plane_batch: int = 0, check_finite: bool = False):
        import torch
        self.torch = torch
        self.w = w
        self.cfg = make_config(w, plane_batch, check_finite)
        h = ctypes.c_void_p()
        _check(library().lmvd_plan_create(ctypes.byref(self.cfg), ctypes.byref(h)), "lmvd_plan_create")
        self.handle = h
        se, ss, wb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(library().lmvd_sizes(h, ctypes.byref(se), ctypes.byref(ss), ctypes.byref(wb)), "lmvd_sizes")
        self.sfield_elems, self.sfield_star_elems, self.workspace_bytes = se.value, ss.value, wb.value
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + self.workspace_bytes]
        self.shape = w.shape
        self.shape_star = w.shape_star

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                library().lmvd_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def factor_check(self, growth_max: float = 0.0):
        """The A(k) pivot check of plan creation (growth_max = 0), or made again with another limit
        (lmvd_factor_check).  Returns (status, max growth, min pivot ratio, failed rows)."""
        g, r, bad = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        st = library().lmvd_factor_check(self.handle, growth_max, ctypes.byref(g), ctypes.byref(r), ctypes.byref(bad))
        if st not in (0, -5):
            _check(st, "lmvd_factor_check")
        return st, g.value, r.value, bad.value

    TILE_CODES = (1, 2, 4, 9, 10, 12, 17, 18, 20)

    def autotune(self, force: int = 0):
        """Pick the z-transform tile (line plan and divisor, code D + 8 V) by timing (force = 0) or set it
        (force = a code); see lmvd_autotune.  Returns (code, per-code ms or -1, in TILE_CODES order)."""
        z = ctypes.c_int32()
        t = (ctypes.c_double * 9)()
        _check(library().lmvd_autotune(self.handle, _ptr(self.ws), self._stream(), force, ctypes.byref(z), t),
               "lmvd_autotune")
        return z.value, list(t)

    # -- helpers ---------------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def empty(self, star=False):
        return self.torch.empty(self.shape_star if star else self.shape, dtype=self.torch.complex128,
                                device="cuda")

    def to_dev(self, a):
        t = self.torch.from_numpy(np.ascontiguousarray(a))
        return t.to("cuda")

    @staticmethod
    def _req(t, dtype):
        if t is None or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
            raise LmvdError("expected a contiguous CUDA tensor of dtype %s" % dtype)

    # -- the substep -------------------------------------------------------------
    def substep(self, stage, phi2, omega2, z, m1bar, m3bar, **kw):
        """One substep; see lmvd.h.  rhs_prev / rhs_out are dicts with keys
        phi2, omega2, m1bar, m3bar.  Outputs default to in-place (except z_out)."""
        a = self.substep_args(stage, phi2, omega2, z, m1bar, m3bar, **kw)
        _check(library().lmvd_substep(self.handle, ctypes.byref(a), _ptr(self.ws), self._stream()),
               "lmvd_substep")

    def substep_args(self, stage, phi2, omega2, z, m1bar, m3bar, *, z_out, phi2_out=None, omega2_out=None,
                     m1bar_out=None, m3bar_out=None, hist=None, kf=-1, guess_mode=0, rhs_prev=None, zt_prev=None,
                     rhs_out=None, zt_out=None, md=None, mc=None):
        """The argument struct of one substep (nothing is launched)."""
        torch = self.torch
        c128, f64 = torch.complex128, torch.float64
        for t in (phi2, omega2, z, z_out):
            self._req(t, c128)
        for t in (m1bar, m3bar):
            self._req(t, f64)
        a = SubstepArgs()
        a.stage, a.kf, a.guess_mode = stage, kf, guess_mode
        a.phi2, a.omega2, a.z = _ptr(phi2), _ptr(omega2), _ptr(z)
        a.m1bar, a.m3bar = _ptr(m1bar), _ptr(m3bar)
        a.phi2_out = _ptr(phi2_out if phi2_out is not None else phi2)
        a.omega2_out = _ptr(omega2_out if omega2_out is not None else omega2)
        a.z_out = _ptr(z_out)
        a.m1bar_out = _ptr(m1bar_out if m1bar_out is not None else m1bar)
        a.m3bar_out = _ptr(m3bar_out if m3bar_out is not None else m3bar)
        if rhs_prev is not None:
            a.rhs_phi2_prev, a.rhs_omega2_prev = _ptr(rhs_prev["phi2"]), _ptr(rhs_prev["omega2"])
            a.rhs_m1_prev, a.rhs_m3_prev = _ptr(rhs_prev["m1bar"]), _ptr(rhs_prev["m3bar"])
        a.zt_prev = _ptr(zt_prev)
        if rhs_out is not None:
            a.rhs_phi2, a.rhs_omega2 = _ptr(rhs_out["phi2"]), _ptr(rhs_out["omega2"])
            a.rhs_m1, a.rhs_m3 = _ptr(rhs_out["m1bar"]), _ptr(rhs_out["m3bar"])
        a.zt = _ptr(zt_out)
        if hist is not None:
            for i in range(3):
                a.z_hist[i] = hist[i].data_ptr()
        if md is not None:
            for i in range(3):
                a.md[i] = md[i].data_ptr()
        if mc is not None:
            for i in range(3):
                a.mc[i] = mc[i].data_ptr()
        return a

    # -- adjoint of the substep ---------------------------------------------------------
    def adjoint_workspace(self, kf: int = -1):
        """The adjoint's workspace (lmvd_adjoint_sizes; it contains the substep's), allocated once per k_f."""
        kf = self.w.kf if kf < 0 else kf
        cache = self.__dict__.setdefault("_adj_ws", {})
        if kf not in cache:
            b = ctypes.c_size_t()
            _check(library().lmvd_adjoint_sizes(self.handle, kf, ctypes.byref(b)), "lmvd_adjoint_sizes")
            buf = self.torch.empty(b.value + 256, dtype=self.torch.uint8, device="cuda")
            off = (-buf.data_ptr()) % 256
            cache[kf] = (buf, buf[off:off + b.value])
        return cache[kf][1]

    def substep_adjoint(self, stage, inputs, cot, kf=-1, guess_mode=0):
        """Gradients of <cot, outputs of one substep> with respect to its inputs (lmvd_substep_adjoint).
        inputs: phi2, omega2, z, m1bar, m3bar, hist (3), and at stage 1 rhs_prev (dict), zt_prev (device
        tensors).  cot: phi2_out, omega2_out, z_out, m1bar_out, m3bar_out, rhs (dict: phi2, omega2,
        m1bar, m3bar), zt, optional md, mc (3-tuples); any missing entry is zero.  Returns a dict like
        inputs with the gradients."""
        torch = self.torch
        w = self.w
        zS = lambda star=False: self.empty(star).zero_()
        zV = lambda: torch.zeros(w.n2, dtype=torch.float64, device="cuda")
        rhs = cot.get("rhs") or {}
        c = {"phi2_out": cot.get("phi2_out"), "omega2_out": cot.get("omega2_out"), "z_out": cot.get("z_out"),
             "m1bar_out": cot.get("m1bar_out"), "m3bar_out": cot.get("m3bar_out"), "rhs_phi2": rhs.get("phi2"),
             "rhs_omega2": rhs.get("omega2"), "zt": cot.get("zt"), "rhs_m1": rhs.get("m1bar"),
             "rhs_m3": rhs.get("m3bar")}
        keep = []
        for k in c:
            if c[k] is None:
                c[k] = zV() if k in ("m1bar_out", "m3bar_out", "rhs_m1", "rhs_m3") else zS()
            c[k] = c[k].contiguous()
            keep.append(c[k])
        g = SubstepGrads()
        for k, v in c.items():
            setattr(g, k, _ptr(v))
        for name in ("md", "mc"):
            t = cot.get(name)
            if t is not None:
                arr = getattr(g, name)
                for i in range(3):
                    if t[i] is not None:
                        x = t[i].contiguous()
                        keep.append(x)
                        arr[i] = x.data_ptr()
        out = {"phi2": zS(), "omega2": zS(), "z": zS(), "m1bar": zV(), "m3bar": zV()}
        for k in ("phi2", "omega2", "z", "m1bar", "m3bar"):
            setattr(g, k, _ptr(out[k]))
        if guess_mode == 0:
            out["hist"] = [zS() for _ in range(3)]
            for i in range(3):
                g.z_hist[i] = out["hist"][i].data_ptr()
        if stage == 1:
            out["rhs_prev"] = {"phi2": zS(), "omega2": zS(), "m1bar": zV(), "m3bar": zV()}
            out["zt_prev"] = zS()
            g.rhs_phi2_prev, g.rhs_omega2_prev = _ptr(out["rhs_prev"]["phi2"]), _ptr(out["rhs_prev"]["omega2"])
            g.rhs_m1_prev, g.rhs_m3_prev = _ptr(out["rhs_prev"]["m1bar"]), _ptr(out["rhs_prev"]["m3bar"])
            g.zt_prev = _ptr(out["zt_prev"])
        a = self.substep_args(stage, inputs["phi2"], inputs["omega2"], inputs["z"], inputs["m1bar"],
                              inputs["m3bar"], z_out=zS(), hist=inputs.get("hist"), kf=kf, guess_mode=guess_mode,
                              rhs_prev=inputs.get("rhs_prev"), zt_prev=inputs.get("zt_prev"))
        _check(library().lmvd_substep_adjoint(self.handle, ctypes.byref(a), ctypes.byref(g),
                                              _ptr(self.adjoint_workspace(kf)), self._stream()),
               "lmvd_substep_adjoint")
        return out

    # -- timing hook -----------------------------------------------------------------
    KERNEL_CLASSES = ("zinv", "xpass_rz", "xpass_l", "xpass_rhot", "xpass_vel", "zfwd", "mc", "md", "proj",
                      "proj_zt", "values", "flux", "rhs", "xpass_io", "zfilt")

    def profile_start(self, cls: int, max_launches: int = 65536):
        _check(library().lmvd_profile_start(self.handle, cls, max_launches), "lmvd_profile_start")

    def profile_stop(self):
        """(total_ms, launches, compulsory_bytes) of the timed kernel class."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(library().lmvd_profile_stop(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
               "lmvd_profile_stop")
        return ms.value, n.value, b.value

    # -- operator entry points ------------------------------------------------------
    def to_physical(self, values):
        w = self.w
        out = self.torch.empty((w.n2, w.m3, w.m1), dtype=self.torch.float64, device="cuda")
        _check(library().lmvd_to_physical(self.handle, _ptr(values), _ptr(out), _ptr(self.ws), self._stream()),
               "lmvd_to_physical")
        return out

    def to_spectral(self, phys):
        out = self.empty()
        _check(library().lmvd_to_spectral(self.handle, _ptr(phys), _ptr(out), _ptr(self.ws), self._stream()),
               "lmvd_to_spectral")
        return out

    def project(self, kind, values):
        out = self.empty()
        _check(library().lmvd_project(self.handle, kind, _ptr(values), _ptr(out), self._stream()), "lmvd_project")
        return out

    def evaluate(self, deriv, coeffs, star=False):
        out = self.empty()
        _check(library().lmvd_evaluate(self.handle, deriv, int(star), _ptr(coeffs), _ptr(out), self._stream()),
               "lmvd_evaluate")
        return out

    # transposes (lmvd_*_adjoint): <A x, y> = <x, A^T y> in the real inner products
    def to_physical_adjoint(self, phys):
        out = self.empty()
        _check(library().lmvd_to_physical_adjoint(self.handle, _ptr(phys), _ptr(out), _ptr(self.ws), self._stream()),
               "lmvd_to_physical_adjoint")
        return out

    def to_spectral_adjoint(self, values):
        w = self.w
        out = self.torch.empty((w.n2, w.m3, w.m1), dtype=self.torch.float64, device="cuda")
        _check(library().lmvd_to_spectral_adjoint(self.handle, _ptr(values), _ptr(out), _ptr(self.ws), self._stream()),
               "lmvd_to_spectral_adjoint")
        return out

    def evaluate_adjoint(self, deriv, values, star=False):
        out = self.empty(star)
        _check(library().lmvd_evaluate_adjoint(self.handle, deriv, int(star), _ptr(values), _ptr(out),
                                               self._stream()), "lmvd_evaluate_adjoint")
        return out

    def project_adjoint(self, kind, coeffs):
        out = self.empty()
        _check(library().lmvd_project_adjoint(self.handle, kind, _ptr(coeffs), _ptr(out), self._stream()),
               "lmvd_project_adjoint")
        return out

    def md_adjoint(self, m1, m2, m3):
        """Transpose of md: adjoints of (m1, m2, m3) -> adjoints of (phi2, Omega2, <m>1, <m>3)."""
        torch = self.torch
        phi, om = self.empty(), self.empty()
        b1 = torch.empty(self.w.n2, dtype=torch.float64, device="cuda")
        b3 = torch.empty(self.w.n2, dtype=torch.float64, device="cuda")
        _check(library().lmvd_md_adjoint(self.handle, _ptr(m1), _ptr(m2), _ptr(m3), _ptr(phi), _ptr(om), _ptr(b1),
                                         _ptr(b3), _ptr(self.ws), self._stream()), "lmvd_md_adjoint")
        return phi, om, b1, b3

    def mc_adjoint(self, m1, m2, m3):
        """Transpose of mc: adjoints of (m1, m2, m3) -> adjoint of rho_t (B coefficients)."""
        out = self.empty()
        _check(library().lmvd_mc_adjoint(self.handle, _ptr(m1), _ptr(m2), _ptr(m3), _ptr(out), _ptr(self.ws),
                                         self._stream()), "lmvd_mc_adjoint")
        return out

    def md(self, phi2, omega2, m1bar, m3bar):
        m1, m2, m3 = self.empty(), self.empty(True), self.empty()
        _check(library().lmvd_md(self.handle, _ptr(phi2), _ptr(omega2), _ptr(m1bar), _ptr(m3bar), _ptr(m1),
                                 _ptr(m2), _ptr(m3), _ptr(self.ws), self._stream()), "lmvd_md")
        return m1, m2, m3

    def mc(self, rhot):
        m1, m2, m3 = self.empty(), self.empty(True), self.empty()
        _check(library().lmvd_mc(self.handle, _ptr(rhot), _ptr(m1), _ptr(m2), _ptr(m3), _ptr(self.ws),
                                 self._stream()), "lmvd_mc")
        return m1, m2, m3

    def rhs(self, z, m1, m2, m3):
        """Right-hand sides of phi2, Omega2 and the plane means for z and m (lmvd_rhs)."""
        torch = self.torch
        rp, ro = self.empty(), self.empty()
        r1 = torch.empty(self.w.n2, dtype=torch.float64, device="cuda")
        r3 = torch.empty(self.w.n2, dtype=torch.float64, device="cuda")
        _check(library().lmvd_rhs(self.handle, _ptr(z), _ptr(m1), _ptr(m2), _ptr(m3), _ptr(rp), _ptr(ro), _ptr(r1),
                                  _ptr(r3), _ptr(self.ws), self._stream()), "lmvd_rhs")
        return {"phi2": rp, "omega2": ro, "m1bar": r1, "m3bar": r3}


class Stepper:
    """Holds the device state of one simulation and advances it by substeps
    (the z history ring, stored RHS and z_t between the two stages)."""

    def __init__(self, plan: Plan, inputs: dict, stage: int = 0):
        torch = plan.torch
        self.p = plan
        dev = plan.to_dev
        self.phi2, self.omega2 = dev(inputs["phi2"]), dev(inputs["omega2"])
        self.z = dev(inputs["z"])
        self.m1bar, self.m3bar = dev(inputs["m1bar"]), dev(inputs["m3bar"])
        self.hist = [dev(h) for h in inputs["hist"]]
        self.stage = stage
        self.rhs = {k: (plan.empty() if k in ("phi2", "omega2") else torch.empty(plan.w.n2, dtype=torch.float64,
                                                                                     device="cuda"))
                    for k in ("phi2", "omega2", "m1bar", "m3bar")}
        self.zt = plan.empty()
        if stage == 1:
            rp = inputs["rhs_prev"]
            for k in self.rhs:
                self.rhs[k].copy_(dev(rp[k]))
            self.zt.copy_(dev(inputs["zt_prev"]))
        self.zt_next = plan.empty()

    # -- checkpoint / resume ------------------------------------------------------
    def save(self, path):
        """Write everything the next substeps read (z and its history ring, phi2, Omega2, the plane
        means, the stage, and at stage ' the stored stage-n RHS and z_t) to a numpy .npz file."""
        torch = self.p.torch
        torch.cuda.synchronize()
        host = lambda t: t.detach().cpu().numpy()
        arrs = {"stage": np.array(self.stage), "z": host(self.z), "phi2": host(self.phi2),
                "omega2": host(self.omega2), "m1bar": host(self.m1bar), "m3bar": host(self.m3bar),
                "zt": host(self.zt)}
        for i, h in enumerate(self.hist):
            arrs[f"hist{i}"] = host(h)
        for k, v in self.rhs.items():
            arrs[f"rhs_{k}"] = host(v)
        np.savez(path, **arrs)

    @classmethod
    def load(cls, plan, path):
        """A Stepper on `plan` resumed from a file written by save(); the plan must have the same sizes."""
        with np.load(path) as d:
            if d["z"].shape != tuple(plan.shape):
                raise LmvdError(f"checkpoint shape {d['z'].shape} does not match the plan's {tuple(plan.shape)}")
            stage = int(d["stage"])
            inputs = {k: d[k] for k in ("phi2", "omega2", "z", "m1bar", "m3bar")}
            inputs["hist"] = [d[f"hist{i}"] for i in range(3)]
            inputs["rhs_prev"] = {k: d[f"rhs_{k}"] for k in ("phi2", "omega2", "m1bar", "m3bar")}
            inputs["zt_prev"] = d["zt"]
        return cls(plan, inputs, stage=stage)

    def next_args(self, kf=-1):
        """Argument struct of the next substep; advances the state bookkeeping
        (history ring, stage) without launching anything."""
        p = self.p
        z_new = self.hist[2]          # the oldest history slot is free after this substep
        if self.stage == 0:
            a = p.substep_args(0, self.phi2, self.omega2, self.z, self.m1bar, self.m3bar, z_out=z_new,
                               hist=self.hist, kf=kf, rhs_out=self.rhs, zt_out=self.zt)
        else:
            a = p.substep_args(1, self.phi2, self.omega2, self.z, self.m1bar, self.m3bar, z_out=z_new,
                               hist=self.hist, kf=kf, rhs_prev=self.rhs, zt_prev=self.zt, zt_out=self.zt_next)
        self.hist = [self.z, self.hist[0], self.hist[1]]
        self.z = z_new
        self.stage = 1 - self.stage
        return a

    def substep(self, kf=-1):
        a = self.next_args(kf)
        _check(library().lmvd_substep(self.p.handle, ctypes.byref(a), _ptr(self.p.ws), self.p._stream()),
               "lmvd_substep")

    def state(self):
        """The state tensors (current z, its history, phi2, Omega2, plane means, stored RHS and z_t)."""
        return dict(z=self.z, hist=list(self.hist), phi2=self.phi2, omega2=self.omega2, m1bar=self.m1bar,
                    m3bar=self.m3bar, rhs=dict(self.rhs), zt=self.zt, zt_next=self.zt_next, stage=self.stage)


class GraphBatch:
    """`nsub` substeps of several independent simulations (Steppers, each with
    its own plan) captured as one HIP graph; launch() advances every one of
    them by nsub substeps.  nsub must be a multiple of 4: the z history ring
    and the stage pattern then repeat, so the baked-in pointers stay valid for
    every launch.  The Steppers must not be advanced otherwise while the graph
    is in use."""

    def __init__(self, steppers, nsub: int = 4, kf=-1):
        """kf: one k_f for all instances, or one per instance (-1 = the plan's)."""
        if nsub % 4 != 0 or not steppers:
            raise LmvdError("GraphBatch: nsub must be a positive multiple of 4")
        self.steppers = list(steppers)
        n = len(self.steppers)
        kfs = list(kf) if isinstance(kf, (list, tuple)) else [kf] * n
        if len(kfs) != n:
            raise LmvdError("GraphBatch: one kf per instance")
        args = (SubstepArgs * (n * nsub))()
        for i, st in enumerate(self.steppers):
            for k in range(nsub):
                args[i * nsub + k] = st.next_args(kfs[i])
        plans = (ctypes.c_void_p * n)(*[st.p.handle.value for st in self.steppers])
        ws = (ctypes.c_void_p * n)(*[st.p.ws.data_ptr() for st in self.steppers])
        h = ctypes.c_void_p()
        _check(library().lmvd_graph_create(plans, args, ws, n, nsub, ctypes.byref(h)), "lmvd_graph_create")
        self.handle = h
        self.nsub = nsub
        self._args, self._plans, self._ws = args, plans, ws

    def autotune(self, launches: int = 3):
        """Pick the z tiles by timing this graph (lmvd_graph_autotune) and capture it again with them.
        Advances every instance like warm-up launches.  Returns (divisor per instance, ms per launch)."""
        n = len(self.steppers)
        torch = self.steppers[0].p.torch
        z = (ctypes.c_int32 * n)()
        ms = ctypes.c_double()
        library().lmvd_graph_destroy(self.handle)
        self.handle = None
        _check(library().lmvd_graph_autotune(self._plans, self._args, self._ws, n, self.nsub,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), launches, z,
                                             ctypes.byref(ms)), "lmvd_graph_autotune")
        h = ctypes.c_void_p()
        _check(library().lmvd_graph_create(self._plans, self._args, self._ws, n, self.nsub, ctypes.byref(h)),
               "lmvd_graph_create")
        self.handle = h
        return list(z), ms.value

    @property
    def grouped(self) -> bool:
        """True when every kernel step is one launch over the instances."""
        v = ctypes.c_int32()
        _check(library().lmvd_graph_grouped(self.handle, ctypes.byref(v)), "lmvd_graph_grouped")
        return bool(v.value)

    def launch(self):
        torch = self.steppers[0].p.torch
        _check(library().lmvd_graph_launch(self.handle, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "lmvd_graph_launch")

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                library().lmvd_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
