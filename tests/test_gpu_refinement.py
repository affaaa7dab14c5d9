"""GPU tests of the bookkeeping around Alg. 1: the residual history cps_get_history returns,
checked against the oracle's residual of the same iterate; the FP64 finish of a
mixed-precision solve whose FP32 refinement is cut short, checked against the oracle's
solution; and the sweep timing, which must count the right sweeps and change nothing."""
import math

import numpy as np
import pytest

import oracle
import paper_1901_08269_amd as cps
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sphere():                       # (40, 40, 40), stretched, one sphere
    return W.sphere_sin(38, beta=1.4, r=0.27, c=(0.52, 0.47, 0.5))


def _two_bodies():                   # (70, 41, 29): unequal sides, a sphere and an ellipsoid
    x, y, z = W.tanh_grid(70, 1.5), W.tanh_grid(41, 1.0), W.uniform_grid(29)
    bodies = [W.Sphere((0.33, 0.45, 0.5), 0.17),
              W.Ellipsoid((0.7, 0.55, 0.48), (0.16, 0.1, 0.2),
                          W._random_rotation(np.random.Generator(np.random.PCG64(5))))]
    return W.polynomial_case(0, bodies, rng_seed=9, grids=(x, y, z))


@pytest.mark.parametrize("precond", ["multigrid", "chebyshev"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_history_covers_every_iteration(precision, precond):
    print(f"[case] history sphere 40^3 {precision} {precond}", flush=True)
    tol = 1e-10
    S = cps.Solver.from_workload(_sphere(), precision=precision, precond=precond)
    _, st = S.solve(tol)
    it, tr = S.history()
    print(f"{st['iters']} iterations, {len(tr)} true residuals, last recursive {it[-1]:.3e}")
    assert len(it) == st["iters"] > 0 and np.all(np.isfinite(it)) and np.all(it > 0)
    # from zero the first true residual is b itself; the last is the one the stats report
    assert abs(tr[0, 0] - 1.0) <= 1e-12 and abs(tr[0, 1] - 1.0) <= 1e-12
    assert tr[-1, 0] == st["rel_residual"] and tr[-1, 1] == st["rel_residual_jacobi"]
    # the recursion stops at a target at most tol (Jacobi-weighted)
    assert it[-1] <= tol * (1 + 1e-9)
    if precision == "mixed":
        # one true residual per refinement step and the final one; every step cut it by > sqrt(2)
        assert len(tr) == st["refine_steps"] + 1
        assert np.all(tr[1:, 1] <= tr[:-1, 1] / math.sqrt(2.0))
    else:
        assert len(tr) == st["restarts"] + 2


def test_history_of_a_truncated_solve_matches_the_oracle_residual():
    """After q iterations (max_iters = q) the last true residual is that of the returned
    iterate, recomputed here by the oracle; the q-th recursive residual of the history equals
    the true one up to FP64 rounding."""
    w = _sphere()
    P = oracle.Problem.from_workload(w)
    for q in (1, 3, 6):
        print(f"[case] truncated fp64 solve, {q} iterations", flush=True)
        S = cps.Solver.from_workload(w, precision="fp64", precond="chebyshev", max_iters=q)
        u, st = S.solve(1e-12, check=False)
        assert st["status"] == cps.CPS_ENOCONV and st["iters"] == q
        it, tr = S.history()
        _, rel = P.residual(u.cpu().numpy())
        print(f"  true {tr[-1, 0]:.6e} (oracle {rel:.6e}), recursive {it[-1]:.6e} vs {tr[-1, 1]:.6e}")
        assert len(it) == q and len(tr) == 2
        assert abs(tr[-1, 0] - rel) <= 1e-9 * rel
        assert abs(it[-1] - tr[-1, 1]) <= 1e-6 * tr[-1, 1]
        S.close()


def test_mixed_solve_finishes_in_fp64_when_refinement_is_cut_short():
    """max_refine = 1: one FP32 refinement step, then FP64 BiCGSTAB from its iterate to the
    tolerance (fp64_finish, the default), with the oracle's solution; without the finish the
    solve reports CPS_ENOCONV after that step."""
    w = _two_bodies()
    print("[case] mixed solve, max_refine 1, two_bodies_aniso", flush=True)
    P = oracle.Problem.from_workload(w)
    u_ref, _ = P.solve(1e-13)
    t = P.types()
    fl = (t == 1) | (t == 2)
    S = cps.Solver.from_workload(w, precision="mixed", max_refine=1)
    u, st = S.solve(1e-12)
    it, tr = S.history()
    rel = np.max(np.abs(u.cpu().numpy() - u_ref)[fl]) / np.max(np.abs(u_ref[fl]))
    print(f"{st['iters_fp32']} FP32 + {st['iters'] - st['iters_fp32']} FP64 iterations, vs oracle {rel:.2e}")
    assert st["refine_steps"] == 1 and 0 < st["iters_fp32"] < st["iters"]
    assert st["rel_residual"] <= 1e-12 and st["rel_residual_jacobi"] <= 1e-12
    assert rel <= 1e-9
    assert len(it) == st["iters"] and len(tr) >= 3
    S0 = cps.Solver.from_workload(w, precision="mixed", max_refine=1, fp64_finish=False)
    _, st0 = S0.solve(1e-12, check=False)
    assert st0["status"] == cps.CPS_ENOCONV and st0["iters"] == st0["iters_fp32"] == st["iters_fp32"]


@pytest.mark.parametrize("precond", ["multigrid", "chebyshev"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_timing_counts_and_leaves_the_solution_unchanged(precision, precond):
    """kernel_timing stamps the smoother sweeps' own start and end on the problem's grid: the
    stats count them, their bytes are 3 vectors per interior point for a pass's first step and
    4 for the others (the full-traffic sweeps, counted apart), and the solve is bitwise the one
    without timing."""
    print(f"[case] sweep timing sphere 40^3 {precision} {precond}", flush=True)
    w = _sphere()
    u0, st0 = cps.Solver.from_workload(w, precision=precision, precond=precond).solve(1e-10)
    u1, st1 = cps.Solver.from_workload(w, precision=precision, precond=precond, kernel_timing=1).solve(1e-10)
    n, nf, pts = st1["sweep_launches"], st1["sweep_full_launches"], st1["sweep_points"]
    vb = 4 if precision == "mixed" else 8
    print(f"{n} timed sweeps ({nf} full-traffic), {1e3 * st1['sweep_ms'] / max(n, 1):.2f} us each")
    assert pts == 38 ** 3 and 0 < nf < n
    assert st1["sweep_bytes"] == (3 * (n - nf) + 4 * nf) * vb * pts
    assert 0.0 < st1["sweep_full_ms"] < st1["sweep_ms"] and 0.0 < st1["sweep_ms"] / n < 5.0
    assert st0["sweep_launches"] == 0 and st0["sweep_ms"] == 0.0
    assert st1["iters"] == st0["iters"] and bool((u0 == u1).all())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_host_pointer_setup_and_solve_match_device_pointers(precision):
    """The C-ABI with host arrays (device_ptrs = 0: the library uploads phi, g and f before
    classifying them, and copies the solution back) gives the solution of the device-array
    path (where the classification pass copies the fields on the way), bit for bit."""
    import ctypes as C
    print(f"[case] host pointers sphere 40^3 {precision}", flush=True)
    w = _sphere()
    u_dev, st_dev = cps.Solver.from_workload(w, precision=precision).solve(1e-10)
    L = cps.load_library()
    o = cps.CpsOptions()
    L.cps_default_options(C.byref(o))
    o.precision = cps.CPS_MIXED if precision == "mixed" else cps.CPS_FP64
    o.device_ptrs = 0
    arr = {k: np.ascontiguousarray(getattr(w, k), dtype=np.float64) for k in ("x", "y", "z", "phi", "g", "f")}
    h = C.c_void_p()
    p = lambda a: C.c_void_p(a.ctypes.data)
    rc = L.cps_setup(C.byref(h), len(arr["x"]), len(arr["y"]), len(arr["z"]), p(arr["x"]), p(arr["y"]),
                     p(arr["z"]), p(arr["phi"]), p(arr["g"]), p(arr["f"]), C.byref(o))
    assert rc == 0
    try:
        u = np.empty(tuple(u_dev.shape))
        st = cps.CpsStats()
        st.struct_size = C.sizeof(cps.CpsStats)
        assert L.cps_solve(h, 1e-10, p(u), 0, C.byref(st)) == 0
    finally:
        L.cps_destroy(h)
    assert st.iters == st_dev["iters"]
    assert np.array_equal(u, u_dev.cpu().numpy())


def test_setup_on_a_side_stream_matches_default_stream():
    """The setup builds the multigrid hierarchy on a second stream of its own, ordered after
    the work the solver's stream has queued: a solver on a non-default torch stream (which
    does not synchronise with the null stream) gives the default-stream solver's irregular
    rows and solution bit for bit."""
    import torch
    print("[case] setup on a side stream, sphere 40^3 mixed", flush=True)
    w = _sphere()
    S0 = cps.Solver.from_workload(w, precision="mixed")
    rows0 = [np.asarray(a).copy() for a in S0.irregular()]
    u0, st0 = S0.solve(1e-10)
    u0 = u0.cpu().numpy()
    S0.close()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        S1 = cps.Solver.from_workload(w, precision="mixed")
        rows1 = [np.asarray(a).copy() for a in S1.irregular()]
        u1, st1 = S1.solve(1e-10)
        side.synchronize()
        u1 = u1.cpu().numpy()
        S1.close()
    assert all(np.array_equal(a, b) for a, b in zip(rows0, rows1))
    assert st1["iters"] == st0["iters"]
    assert np.array_equal(u1, u0)
