"""The C-ABI library loads on a machine without a GPU and exports every function that
include/cps.h declares (no compute calls here)."""
import ctypes
import os

import pytest

import paper_1901_08269_amd as cps


def test_header_declares_core_entry_points():
    names = cps.header_symbols()
    for required in ("cps_setup", "cps_solve", "cps_residual", "cps_apply", "cps_precond", "cps_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(cps.LIB_PATH), reason="libcps.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(cps.LIB_PATH)
    missing = [n for n in cps.header_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(cps.LIB_PATH), reason="libcps.so not built")
def test_struct_layouts_and_host_only_calls():
    lib = cps.load_library()
    o = cps.CpsOptions()
    lib.cps_default_options(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(cps.CpsOptions) == 104
    assert o.inner_iters == 24 and o.precision == cps.CPS_FP64
    assert o.precond == cps.CPS_PRECOND_MULTIGRID
    assert (o.mg_levels, o.mg_nu, o.mg_coarse_steps, o.mg_smooth_lo) == (16, 2, 8, 0.2)
    assert (o.sip_iters, o.sip_alpha) == (8, 0.9)
    assert o.fp64_finish == 1 and o.max_refine == 40
    # lam_lo = 0 selects max(lam_hi / (4 inner_iters^2), lambda_1 of the grid) at setup
    assert abs(o.inner_tol - 1e-4) < 1e-18 and o.lam_hi == 2.0 and o.lam_lo == 0.0
    assert lib.cps_strerror(-2).decode().startswith("invalid geometry")
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert lib.cps_setup(ctypes.byref(h), 2, 5, 5, None, None, None, None, None, None, None) == -1
    # the history query validates its arguments before touching the solver
    n = ctypes.c_int32()
    assert lib.cps_get_history(None, None, 0, ctypes.byref(n), None, 0, None) == -1


@pytest.mark.skipif(not os.path.exists(cps.LIB_PATH), reason="libcps.so not built")
def test_multigrid_options_validated_before_device_calls():
    """Out-of-range preconditioner settings are rejected (CPS_EINVAL) before any HIP call."""
    import numpy as np
    lib = cps.load_library()
    n = 6
    x = np.linspace(0.0, 1.0, n)
    a = np.ones((n, n, n))
    dp = lambda arr: arr.ctypes.data_as(ctypes.c_void_p)
    bad = [("precond", 3), ("precond", -1), ("mg_levels", 0), ("mg_levels", 17), ("mg_nu", 0), ("mg_nu", 65),
           ("mg_coarse_steps", 0), ("mg_smooth_lo", 0.0), ("mg_smooth_lo", 2.0), ("sip_iters", 0),
           ("sip_iters", 65), ("sip_alpha", -0.5), ("sip_alpha", 1.01), ("fp64_finish", 2),
           ("fp64_finish", -1)]
    for name, val in bad:
        o = cps.CpsOptions()
        lib.cps_default_options(ctypes.byref(o))
        o.precond = cps.CPS_PRECOND_MULTIGRID
        setattr(o, name, val)
        h = ctypes.c_void_p()
        rc = lib.cps_setup(ctypes.byref(h), n, n, n, dp(x), dp(x), dp(x), dp(a), dp(a), dp(a), ctypes.byref(o))
        assert rc == -1, (name, val, rc)
