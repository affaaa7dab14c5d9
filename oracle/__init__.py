"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU oracle (cps_oracle.c).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never loads it and shares no code with it.

Every function documents the passage of the paper it follows in the C source.  The
network oracle (net_oracle.c) is wrapped in oracle.net.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libcps_oracle.so")
_SRCS = ["cps_oracle.c", "net_oracle.c"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain C, no SIMD intrinsics, no FMA contraction)."""
    os.makedirs(_BUILD, exist_ok=True)
    srcs = [os.path.join(_HERE, s) for s in _SRCS if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_int)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_info.argtypes = [C.c_void_p, C.POINTER(C.c_longlong)]
        L.orc_min_hb.restype = C.c_double
        L.orc_min_hb.argtypes = [C.c_void_p]
        L.orc_types.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_rhs.argtypes = [C.c_void_p, dp]
        L.orc_irregular_nodes.argtypes = [C.c_void_p, C.POINTER(C.c_longlong)]
        L.orc_row.restype = C.c_int
        L.orc_row.argtypes = [C.c_void_p, C.c_longlong, C.POINTER(C.c_longlong), dp, C.c_int]
        L.orc_krow.restype = C.c_int
        L.orc_krow.argtypes = [C.c_void_p, C.c_longlong, dp]
        L.orc_apply.argtypes = [C.c_void_p, dp, dp]
        L.orc_apply_K.argtypes = [C.c_void_p, dp, dp]
        L.orc_precond.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_double, C.c_double]
        L.orc_smooth.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_double, C.c_double]
        L.orc_create_k.restype = C.c_void_p
        L.orc_create_k.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, C.POINTER(C.c_int)]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [C.c_void_p, C.c_double, dp, C.c_void_p, dp]
        L.orc_residual.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_compact_coef.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_second_coef.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_sip_factor.argtypes = [C.c_void_p, C.c_double, dp]
        L.orc_sip_precond.argtypes = [C.c_void_p, dp, dp, dp, C.c_int]
        L.orc_onesided_weights.restype = C.c_int
        L.orc_onesided_weights.argtypes = [C.c_int, dp, C.c_int, dp, dp, C.c_double, C.c_double, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OrcOpts(C.Structure):
    _fields_ = [("inner_iters", C.c_int), ("max_iters", C.c_int), ("mixed", C.c_int),
                ("max_refine", C.c_int), ("max_restarts", C.c_int),
                ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("inner_tol", C.c_double)]


# Default preconditioner parameters, the same policy as the GPU library's defaults (stated
# there independently): 24 Chebyshev-Jacobi steps on [lo, hi] with hi = 2 (Gershgorin bound
# of the diagonally dominant rows of K) and, unless given, lo = max(hi / (4 m^2), lambda_1),
# lambda_1 being the smallest eigenvalue of the Jacobi-scaled 7-point Laplacian on a uniform
# grid with the same point counts n_d: (1/3) sum_d (1 - cos(pi / (n_d - 1))).
DEFAULT_INNER = 24
DEFAULT_LAM_HI = 2.0


def default_lam_lo(m, shape, hi=DEFAULT_LAM_HI):
    lam1 = sum(1.0 - np.cos(np.pi / (n - 1)) for n in shape) / 3.0
    return max(hi / (4.0 * m * m), lam1)


def compact_coef(x):
    x = _f64(x)
    n = len(x)
    out = [np.zeros(n) for _ in range(5)]
    lib().orc_compact_coef(n, _p(x), *[_p(o) for o in out])
    return tuple(out)  # a, c, ar, br, cr


def second_coef(x):
    x = _f64(x)
    n = len(x)
    out = [np.zeros(n) for _ in range(3)]
    lib().orc_second_coef(n, _p(x), *[_p(o) for o in out])
    return tuple(out)  # a, b, c


def onesided_weights(tp, tr, Lw, tref=None, href=None):
    tp, tr, Lw = _f64(tp), _f64(tr), _f64(Lw)
    if tref is None:
        tref = float(tr[0])
    if href is None:
        href = float(np.max(np.abs(tp - tref)))
    w = np.zeros(len(tp))
    rc = lib().orc_onesided_weights(len(tp), _p(tp), len(tr), _p(tr), _p(Lw), tref, href, _p(w))
    if rc != 0:
        raise RuntimeError("singular one-sided system")
    return w


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


class Problem:
    """The discretised problem B u = q + b on one grid and geometry (FP64, CPU)."""

    def __init__(self, x, y, z, phi, g, f):
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        self.shape = (len(self.z), len(self.y), len(self.x))
        self._phi, self._g, self._f = _f64(phi), _f64(g), _f64(f)
        assert self._phi.size == self._g.size == self._f.size == int(np.prod(self.shape))
        err = C.c_int(0)
        self.h = lib().orc_create(len(self.x), len(self.y), len(self.z), _p(self.x), _p(self.y), _p(self.z),
                                  _p(self._phi), _p(self._g), _p(self._f), C.byref(err))
        if not self.h:
            raise OracleError(err.value)

    @classmethod
    def from_workload(cls, w):
        return cls(w.x, w.y, w.z, w.phi, w.g, w.f)

    @classmethod
    def k_only(cls, x, y, z, phi):
        """The grid, node types and K rows only (a coarse level of the multigrid preconditioner)."""
        self = cls.__new__(cls)
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        self.shape = (len(self.z), len(self.y), len(self.x))
        self._phi = _f64(phi)
        err = C.c_int(0)
        self.h = lib().orc_create_k(len(self.x), len(self.y), len(self.z), _p(self.x), _p(self.y), _p(self.z),
                                    _p(self._phi), C.byref(err))
        if not self.h:
            raise OracleError(err.value)
        return self

    def smooth(self, rho, x, iters, lo, hi):
        """`iters` Chebyshev-Jacobi steps on K x = rho from x, spectrum interval [lo, hi]."""
        out = _f64(x).copy()
        lib().orc_smooth(self.h, _p(_f64(rho)), _p(out), iters, lo, hi)
        return out

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    @property
    def nn(self):
        return int(np.prod(self.shape))

    def info(self):
        out = (C.c_longlong * 5)()
        lib().orc_info(self.h, out)
        return {"n_unknown": out[0], "n_irregular": out[1], "n_solid": out[2], "fallback_lines": out[3],
                "nnz_irregular": out[4], "min_hb": lib().orc_min_hb(self.h)}

    def types(self):
        t = np.zeros(self.shape, dtype=np.int8)
        lib().orc_types(self.h, t.ctypes.data_as(C.c_void_p))
        return t

    def rhs(self):
        b = np.zeros(self.shape)
        lib().orc_rhs(self.h, _p(b))
        return b

    def irregular_nodes(self):
        n = self.info()["n_irregular"]
        out = np.zeros(n, dtype=np.int64)
        if n:
            lib().orc_irregular_nodes(self.h, out.ctypes.data_as(C.POINTER(C.c_longlong)))
        return out

    def row(self, node):
        cols = np.zeros(512, dtype=np.int64)
        vals = np.zeros(512)
        cnt = lib().orc_row(self.h, int(node), cols.ctypes.data_as(C.POINTER(C.c_longlong)), _p(vals), 512)
        if cnt < 0:
            raise ValueError("not an unknown node")
        order = np.argsort(cols[:cnt])
        return cols[:cnt][order], vals[:cnt][order]

    def krow(self, node):
        co = np.zeros(7)
        if lib().orc_krow(self.h, int(node), _p(co)) < 0:
            raise ValueError("not an unknown node")
        return co

    def apply(self, x):
        x = _f64(x).reshape(self.shape)
        y = np.zeros(self.shape)
        lib().orc_apply(self.h, _p(x), _p(y))
        return y

    def apply_K(self, x):
        x = _f64(x).reshape(self.shape)
        y = np.zeros(self.shape)
        lib().orc_apply_K(self.h, _p(x), _p(y))
        return y

    def precond(self, rho, iters=DEFAULT_INNER, lo=None, hi=DEFAULT_LAM_HI):
        lo = default_lam_lo(iters, self.shape, hi) if lo is None else lo
        rho = _f64(rho).reshape(self.shape)
        phi = np.zeros(self.shape)
        lib().orc_precond(self.h, _p(rho), _p(phi), iters, lo, hi)
        return phi

    def sip_factors(self, alpha):
        """Factors of the strongly implicit procedure for K: array (7,) + shape holding b, c,
        d, e, f, g, h per node (see orc_sip_factor)."""
        F = np.zeros(self.shape + (7,))
        lib().orc_sip_factor(self.h, float(alpha), _p(F))
        return np.moveaxis(F, -1, 0).copy()

    def precond_sip(self, rho, iters=8, alpha=0.5, factors=None):
        """`iters` iterations of the strongly implicit procedure on K phi = rho from 0."""
        F = self.sip_factors(alpha) if factors is None else factors
        Fn = np.ascontiguousarray(np.moveaxis(F, 0, -1))
        rho = _f64(rho).reshape(self.shape)
        phi = np.zeros(self.shape)
        lib().orc_sip_precond(self.h, _p(Fn), _p(rho), _p(phi), int(iters))
        return phi

    def solve(self, tol=1e-10, u0=None, mixed=False, inner_iters=DEFAULT_INNER, max_iters=20000,
              lam_lo=None, lam_hi=DEFAULT_LAM_HI, inner_tol=1e-4, max_refine=30, max_restarts=5,
              check=True):
        lam_lo = default_lam_lo(inner_iters, self.shape, lam_hi) if lam_lo is None else lam_lo
        u = np.zeros(self.shape) if u0 is None else _f64(u0).reshape(self.shape).copy()
        o = OrcOpts(inner_iters, max_iters, int(mixed), max_refine, max_restarts, lam_lo, lam_hi, inner_tol)
        st = np.zeros(5)
        rc = lib().orc_solve(self.h, tol, _p(u), C.byref(o), _p(st))
        stats = {"iters": int(st[0]), "refine_steps": int(st[1]), "restarts": int(st[2]),
                 "rel_residual": float(st[3]), "rel_residual_jacobi": float(st[4]), "status": rc}
        if check and rc != 0:
            raise OracleError(rc)
        return u, stats

    def residual(self, u):
        u = _f64(u).reshape(self.shape)
        r = np.zeros(self.shape)
        rel = C.c_double(0)
        lib().orc_residual(self.h, _p(u), _p(r), C.byref(rel))
        return r, rel.value

    def csr(self):
        """Assemble B over the unknowns (scipy CSR) and the unknown node list; tiny grids only."""
        import scipy.sparse as sp
        t = self.types().ravel()
        unk = np.nonzero((t == 1) | (t == 2))[0]
        pos = -np.ones(self.nn, dtype=np.int64)
        pos[unk] = np.arange(len(unk))
        rows, cols, vals = [], [], []
        for r, node in enumerate(unk):
            c, v = self.row(node)
            rows.append(np.full(len(c), r))
            cols.append(pos[c])
            vals.append(v)
        B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(len(unk), len(unk)))
        return B, unk
