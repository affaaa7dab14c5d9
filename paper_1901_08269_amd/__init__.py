"""MI355X (gfx950) compact immersed-interface Poisson solver -- Python binding.

A thin ctypes layer over the C-ABI of include/cps.h (libcps.so, built in-tree by
paper_1901_08269_amd.build).  It only marshals arguments: every step of setup and solve
runs in the library's HIP kernels.  PyTorch provides device memory (float64 tensors whose
data_ptr() is handed to the library) and the stream the library launches on.

There is no CPU fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libcps.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cps.h")

CPS_FP64 = 0
CPS_MIXED = 1
CPS_PRECOND_CHEBYSHEV = 0
CPS_PRECOND_MULTIGRID = 1
CPS_PRECOND_SIP = 2
CPS_OK, CPS_EINVAL, CPS_EGEOM, CPS_ENOMEM, CPS_EDEVICE, CPS_EBREAKDOWN, CPS_ENOCONV, CPS_ENAN = 0, -1, -2, -3, -4, -5, -6, -7
ERRORS = {0: "ok", -1: "EINVAL", -2: "EGEOM", -3: "ENOMEM", -4: "EDEVICE", -5: "EBREAKDOWN", -6: "ENOCONV",
          -7: "ENAN"}


class CpsOptions(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("precision", C.c_int32), ("inner_iters", C.c_int32),
                ("max_iters", C.c_int32), ("max_refine", C.c_int32), ("max_restarts", C.c_int32),
                ("device_ptrs", C.c_int32), ("kernel_timing", C.c_int32), ("inner_tol", C.c_double),
                ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("stream", C.c_void_p),
                ("precond", C.c_int32), ("mg_levels", C.c_int32), ("mg_nu", C.c_int32),
                ("mg_coarse_steps", C.c_int32), ("mg_smooth_lo", C.c_double), ("sip_iters", C.c_int32),
                ("fp64_finish", C.c_int32), ("sip_alpha", C.c_double)]


class CpsStats(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("iters", C.c_int32), ("iters_fp32", C.c_int32),
                ("refine_steps", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("n_unknowns", C.c_int64), ("n_irregular", C.c_int64), ("n_solid", C.c_int64),
                ("nnz_irregular", C.c_int64), ("fallback_lines", C.c_int64),
                ("rel_residual", C.c_double), ("rel_residual_jacobi", C.c_double), ("min_ibi_frac", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("sweep_ms", C.c_double),
                ("sweep_launches", C.c_int64), ("sweep_points", C.c_int64), ("sweep_bytes", C.c_double),
                ("sweep_full_ms", C.c_double), ("sweep_full_launches", C.c_int64), ("warm_alpha", C.c_double)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "struct_size"}


class CpsError(RuntimeError):
    def __init__(self, code, where=""):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code})")
        self.code = code


_lib = None


def header_symbols():
    """Names of every function declared in include/cps.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cps_[a-z_0-9]+)\s*\(", text)))


def load_library(path: str = LIB_PATH):
    """Load libcps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1901_08269_amd.build`")
    # torch first: it ships its own HIP runtime, and the library must bind to that same one,
    # or pointers and streams torch hands over belong to a runtime the library does not use
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, dp, i32 = C.c_void_p, C.c_void_p, C.c_int32
    L.cps_default_options.argtypes = [C.POINTER(CpsOptions)]
    L.cps_setup.argtypes = [C.POINTER(vp), i32, i32, i32, dp, dp, dp, dp, dp, dp, C.POINTER(CpsOptions)]
    L.cps_set_rhs.argtypes = [vp, dp, dp]
    L.cps_solve.argtypes = [vp, C.c_double, dp, i32, C.POINTER(CpsStats)]
    L.cps_residual.argtypes = [vp, dp, dp, dp]
    L.cps_apply.argtypes = [vp, dp, dp, i32]
    L.cps_precond.argtypes = [vp, dp, dp, i32]
    L.cps_get_rhs.argtypes = [vp, dp, dp]
    L.cps_get_info.argtypes = [vp, C.POINTER(C.c_int64)]
    L.cps_get_irregular.argtypes = [vp, dp, dp, dp, dp, dp]
    pi32 = C.POINTER(C.c_int32)
    L.cps_get_history.argtypes = [vp, dp, i32, pi32, dp, i32, pi32]
    L.cps_destroy.argtypes = [vp]
    L.cps_strerror.restype = C.c_char_p
    L.cps_strerror.argtypes = [C.c_int]
    for name in ("cps_setup", "cps_set_rhs", "cps_solve", "cps_residual", "cps_apply", "cps_precond", "cps_get_rhs",
                 "cps_get_info", "cps_get_irregular", "cps_get_history"):
        getattr(L, name).restype = C.c_int
    L.cps_destroy.restype = None
    _lib = L
    return L


def default_options():
    """The library's default cps_options (lam_lo = 0 means hi / (4 inner_iters^2))."""
    o = CpsOptions()
    load_library().cps_default_options(C.byref(o))
    return o


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the solver runs only on the MI355X device")
    return torch


def _dev64(a, shape=None):
    torch = _torch()
    t = torch.as_tensor(a, dtype=torch.float64)
    t = t.to("cuda").contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Solver:
    """One discrete problem (grid, bodies, f, g) resident on the GPU.

    Arrays are (nz, ny, nx) float64 (numpy or torch); node (i,j,k) is element [k, j, i].
    """

    def __init__(self, x, y, z, phi, g, f, precision="fp64", inner_iters=None, lam_lo=None, lam_hi=None,
                 inner_tol=1e-4, max_iters=20000, max_refine=40, max_restarts=5, kernel_timing=False,
                 precond=None, mg_levels=None, mg_nu=None, mg_coarse_steps=None, mg_smooth_lo=None,
                 sip_iters=None, sip_alpha=None, fp64_finish=None):
        torch = _torch()
        L = load_library()
        self.L = L
        self.shape = (len(z), len(y), len(x))
        o = CpsOptions()
        L.cps_default_options(C.byref(o))
        o.precision = CPS_MIXED if precision == "mixed" else CPS_FP64
        if inner_iters is not None:
            o.inner_iters = inner_iters
        if lam_lo is not None:
            o.lam_lo = lam_lo
        if lam_hi is not None:
            o.lam_hi = lam_hi
        o.inner_tol = inner_tol
        o.max_iters = max_iters
        o.max_refine = max_refine
        o.max_restarts = max_restarts
        o.kernel_timing = int(kernel_timing)   # True: every sweep; n: every n-th
        if precond is not None:                # "chebyshev", "multigrid" or "sip"
            o.precond = {"chebyshev": CPS_PRECOND_CHEBYSHEV, "multigrid": CPS_PRECOND_MULTIGRID,
                         "sip": CPS_PRECOND_SIP}[precond]
        for name, val in (("mg_levels", mg_levels), ("mg_nu", mg_nu), ("mg_coarse_steps", mg_coarse_steps),
                          ("mg_smooth_lo", mg_smooth_lo), ("sip_iters", sip_iters), ("sip_alpha", sip_alpha),
                          ("fp64_finish", None if fp64_finish is None else int(fp64_finish))):
            if val is not None:
                setattr(o, name, val)
        o.device_ptrs = 1
        self.stream = torch.cuda.current_stream()
        o.stream = C.c_void_p(self.stream.cuda_stream)
        self.opts = o
        xs, ys, zs = _dev64(x), _dev64(y), _dev64(z)
        ph, gg, ff = _dev64(phi, self.shape), _dev64(g, self.shape), _dev64(f, self.shape)
        h = C.c_void_p()
        rc = L.cps_setup(C.byref(h), len(x), len(y), len(z), _ptr(xs), _ptr(ys), _ptr(zs), _ptr(ph), _ptr(gg),
                         _ptr(ff), C.byref(o))
        if rc != 0:
            raise CpsError(rc, "cps_setup")
        self.h = h

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.x, w.y, w.z, w.phi, w.g, w.f, **kw)

    def close(self):
        if getattr(self, "h", None):
            self.L.cps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, where):
        if rc != 0:
            raise CpsError(rc, where)

    def set_rhs(self, f, g):
        ff, gg = _dev64(f, self.shape), _dev64(g, self.shape)
        self._check(self.L.cps_set_rhs(self.h, _ptr(ff), _ptr(gg)), "cps_set_rhs")

    def solve(self, tol=1e-10, u0=None, check=True, out=None, inplace=False):
        """Solve to `tol`; returns (u, stats).  u0: optional warm start.  out: optional
        (nz, ny, nx) float64 CUDA tensor for the solution.  inplace: solve in u0's own storage
        (u0 must then be a contiguous float64 CUDA tensor of the grid's shape; it is
        overwritten by the solution), sparing a copy."""
        torch = _torch()
        warm = 0
        if u0 is not None and inplace:
            if not (torch.is_tensor(u0) and u0.is_cuda and u0.dtype == torch.float64 and u0.is_contiguous()
                    and tuple(u0.shape) == self.shape):
                raise ValueError("inplace needs u0 as a contiguous float64 CUDA tensor of the grid's shape")
            out, warm = u0, 1
        else:
            if out is None:   # the library writes every node
                out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
            if u0 is not None:
                out.copy_(_dev64(u0, self.shape))
                warm = 1
        st = CpsStats()
        st.struct_size = C.sizeof(CpsStats)
        rc = self.L.cps_solve(self.h, tol, _ptr(out), warm, C.byref(st))
        stats = st.to_dict()
        stats["status_name"] = ERRORS.get(rc, rc)
        if check and rc != 0:
            raise CpsError(rc, "cps_solve")
        return out, stats

    def history(self):
        """Residual history of the last solve (numpy): the recursive ||D^-1 r|| / ||D^-1 b||
        after every BiCGSTAB iteration, and the true (||r|| / ||b||, ||D^-1 r|| / ||D^-1 b||)
        before every restart pass or refinement step and at the end (shape (n, 2))."""
        import numpy as np
        ni, nt = C.c_int32(), C.c_int32()
        self._check(self.L.cps_get_history(self.h, None, 0, C.byref(ni), None, 0, C.byref(nt)), "cps_get_history")
        it = np.zeros(max(ni.value, 1))
        tr = np.zeros((max(nt.value, 1), 2))
        self._check(self.L.cps_get_history(self.h, it.ctypes.data, ni.value, C.byref(ni), tr.ctypes.data, nt.value,
                                           C.byref(nt)), "cps_get_history")
        return it[:ni.value], tr[:nt.value]

    def residual(self, u):
        torch = _torch()
        uu = _dev64(u, self.shape)
        r = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        rel = (C.c_double * 2)()
        self._check(self.L.cps_residual(self.h, _ptr(uu), _ptr(r), C.cast(rel, C.c_void_p)), "cps_residual")
        return r, rel[0], rel[1]

    def apply(self, x, precision="fp64"):
        torch = _torch()
        xx = _dev64(x, self.shape)
        y = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        p = CPS_MIXED if precision in ("fp32", "mixed") else CPS_FP64
        self._check(self.L.cps_apply(self.h, _ptr(xx), _ptr(y), p), "cps_apply")
        return y

    def precond(self, rho, precision="fp64"):
        torch = _torch()
        rr = _dev64(rho, self.shape)
        y = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        p = CPS_MIXED if precision in ("fp32", "mixed") else CPS_FP64
        self._check(self.L.cps_precond(self.h, _ptr(rr), _ptr(y), p), "cps_precond")
        return y

    def rhs_and_types(self):
        torch = _torch()
        b = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        t = torch.zeros(self.shape, dtype=torch.int8, device="cuda")
        self._check(self.L.cps_get_rhs(self.h, _ptr(b), _ptr(t)), "cps_get_rhs")
        return b, t

    def info(self):
        out = (C.c_int64 * 6)()
        self._check(self.L.cps_get_info(self.h, out), "cps_get_info")
        return {"n_unknown": out[0], "n_irregular": out[1], "n_solid": out[2], "nnz_irregular": out[3],
                "fallback_lines": out[4], "nn": out[5]}

    def irregular(self):
        """Host copies (numpy) of the irregular rows: node, ptr, col, val, krow."""
        import numpy as np
        inf = self.info()
        n, nnz = inf["n_irregular"], inf["nnz_irregular"]
        node = np.zeros(max(n, 1), np.int64)
        ptr = np.zeros(n + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int64)
        val = np.zeros(max(nnz, 1))
        krow = np.zeros(max(7 * n, 1))
        self._check(self.L.cps_get_irregular(self.h, node.ctypes.data, ptr.ctypes.data, col.ctypes.data,
                                             val.ctypes.data, krow.ctypes.data), "cps_get_irregular")
        return node[:n], ptr, col[:nnz], val[:nnz], krow[:7 * n].reshape(n, 7)
