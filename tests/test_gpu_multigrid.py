"""GPU parity of the multigrid preconditioner for K (one V-cycle per apply) against the
oracle's V-cycle, on the same seeded inputs, in FP64 and FP32, and solves with it."""
import functools

import numpy as np
import pytest

import oracle
import paper_1901_08269_amd as cps
from oracle import mg
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _case(name):
    if name == "sphere_stretched":        # 40^3: three levels (40, 21, 11), the last in one workgroup
        w = W.sphere_sin(38, beta=1.4, r=0.27, c=(0.52, 0.47, 0.5))
    elif name == "two_bodies_aniso":      # (70, 41, 29): two levels
        x, y, z = W.tanh_grid(70, 1.5), W.tanh_grid(41, 1.0), W.uniform_grid(29)
        bodies = [W.Sphere((0.33, 0.45, 0.5), 0.17),
                  W.Ellipsoid((0.7, 0.55, 0.48), (0.16, 0.1, 0.2),
                              W._random_rotation(np.random.Generator(np.random.PCG64(5))))]
        w = W.polynomial_case(0, bodies, rng_seed=9, grids=(x, y, z))
    elif name == "wide_ragged":           # (283, 70, 45): two 256-node row segments, odd and
        # even point counts, three levels (283 -> 142 -> 72 in x)
        x, y, z = W.tanh_grid(283, 1.3), W.tanh_grid(70, 0.9), W.uniform_grid(45)
        bodies = [W.Sphere((0.3, 0.5, 0.5), 0.2), W.Sphere((0.72, 0.42, 0.55), 0.14)]
        w = W.polynomial_case(0, bodies, rng_seed=21, grids=(x, y, z))
    elif name == "ragged_lds":            # (44, 37, 35) -> (23, 19, 18) -> (12, 10, 10): the coarsest
        # grid (640 interior points) is solved in one workgroup
        x, y, z = W.tanh_grid(44, 1.2), W.uniform_grid(37), W.tanh_grid(35, 0.8)
        bodies = [W.Ellipsoid((0.48, 0.52, 0.5), (0.22, 0.15, 0.18),
                              W._random_rotation(np.random.Generator(np.random.PCG64(8))))]
        w = W.polynomial_case(0, bodies, rng_seed=5, grids=(x, y, z))
    elif name == "single_level":          # (300, 14, 11): too small to coarsen
        x, y, z = W.tanh_grid(300, 1.1), W.uniform_grid(14), W.uniform_grid(11)
        w = W.polynomial_case(0, [W.Sphere((0.78, 0.5, 0.47), 0.22)], rng_seed=11, grids=(x, y, z))
    else:
        raise KeyError(name)
    return w


@functools.lru_cache(maxsize=None)
def _oracle_solution(name):
    P = oracle.Problem.from_workload(_case(name))
    u_ref, _ = P.solve(1e-13)
    return P.types(), u_ref


def _random_rho(phi_shape, types, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(phi_shape) * ((types == 1) | (types == 2))


@pytest.mark.parametrize("name", ["sphere_stretched", "two_bodies_aniso", "wide_ragged", "ragged_lds", "single_level"])
def test_vcycle_matches_oracle(name):
    w = _case(name)
    print(f"[case] multigrid {name} shape {w.phi.shape}", flush=True)
    M = mg.Multigrid(w.x, w.y, w.z, w.phi)          # default levels, 2 + 2 steps, 8 coarse
    rho = _random_rho(w.phi.shape, M.lv[0]["P"].types(), 31)
    ref = M.apply(rho)
    scale = np.max(np.abs(ref))
    S = cps.Solver.from_workload(w, precond="multigrid")
    got = _np(S.precond(rho, "fp64"))
    err = np.max(np.abs(got - ref)) / scale
    print(f"levels {len(M.lv)}: fp64 {err:.2e}")
    assert err <= 1e-11
    got32 = _np(S.precond(rho, "fp32"))
    err32 = np.max(np.abs(got32 - ref)) / scale
    print(f"fp32 {err32:.2e}")
    assert err32 <= 2e-5
    # a fixed linear map, applied deterministically
    again = _np(S.precond(rho, "fp64"))
    assert np.array_equal(again, got)
    got2 = _np(S.precond(2.0 * rho, "fp64"))
    assert np.max(np.abs(got2 - 2.0 * got)) <= 1e-12 * scale


def test_vcycle_options_match_oracle():
    """Two levels, one smoothing step each side, 8 coarse steps, smoother interval [0.3, 2]."""
    w = _case("sphere_stretched")
    M = mg.Multigrid(w.x, w.y, w.z, w.phi, levels=2, nu=1, smooth_lo=0.3, coarse_steps=8)
    rho = _random_rho(w.phi.shape, M.lv[0]["P"].types(), 7)
    ref = M.apply(rho)
    S = cps.Solver.from_workload(w, precond="multigrid", mg_levels=2, mg_nu=1, mg_smooth_lo=0.3, mg_coarse_steps=8)
    got = _np(S.precond(rho, "fp64"))
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_one_level_is_the_chebyshev_iteration():
    """With one level the cycle is mg_coarse_steps Chebyshev-Jacobi steps on [lambda_1, 2]:
    the same map as the Chebyshev preconditioner with that interval."""
    w = _case("sphere_stretched")
    lam1 = mg.lambda_1(w.phi.shape)
    Sm = cps.Solver.from_workload(w, precond="multigrid", mg_levels=1, mg_coarse_steps=12)
    Sc = cps.Solver.from_workload(w, inner_iters=12, lam_lo=lam1, precond="chebyshev")
    P = oracle.Problem.k_only(w.x, w.y, w.z, w.phi)
    rho = _random_rho(w.phi.shape, P.types(), 3)
    a, b = _np(Sm.precond(rho, "fp64")), _np(Sc.precond(rho, "fp64"))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["sphere_stretched", "wide_ragged", "ragged_lds"])
def test_solve_with_multigrid_matches_oracle(name, precision):
    w = _case(name)
    print(f"[case] multigrid solve {name} {precision}", flush=True)
    t, u_ref = _oracle_solution(name)
    fl = (t == 1) | (t == 2)
    S = cps.Solver.from_workload(w, precision=precision, precond="multigrid")
    u, st = S.solve(1e-11)
    Sc = cps.Solver.from_workload(w, precision=precision, precond="chebyshev")
    _, stc = Sc.solve(1e-11)
    print(f"iterations: multigrid {st['iters']}, chebyshev {stc['iters']}")
    assert st["rel_residual"] <= 1e-11 and st["rel_residual_jacobi"] <= 1e-11
    u = _np(u)
    rel = np.max(np.abs(u - u_ref)[fl]) / np.max(np.abs(u_ref[fl]))
    assert rel <= 1e-9, rel
    assert np.all(u[t == 3] == 0.0)


def test_spheres8_256_multigrid_vs_oracle_samples():
    """256^3 with 8 spheres, the multigrid preconditioner, both precisions: at tol 1e-10 the
    residual bounds hold; at tol 1e-13 the solution matches the stored FP64 oracle solution
    (solved to 1e-13) to <= 1e-9 relative max-norm on the sampled nodes."""
    from test_gpu_parity import _samples
    nodes, vals, umax = _samples("oracle_spheres8_256.txt")
    w = W.spheres8(256)
    for precision in ("mixed", "fp64"):
        print(f"[case] spheres8 256 multigrid {precision}", flush=True)
        S = cps.Solver.from_workload(w, precision=precision, precond="multigrid")
        u, st = S.solve(1e-10)
        assert st["rel_residual"] <= 1e-10 and st["rel_residual_jacobi"] <= 1e-10
        u, st = S.solve(1e-13)
        assert st["rel_residual"] <= 1e-13 and st["rel_residual_jacobi"] <= 1e-13
        rel = np.max(np.abs(_np(u).ravel()[nodes] - vals)) / umax
        print(f"{precision}: {st['iters']} iterations, max rel. difference vs oracle samples {rel:.2e}")
        assert rel <= 1e-9
        S.close()
