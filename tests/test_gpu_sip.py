"""GPU parity of the strongly implicit procedure for K (the preconditioner option "sip",
hyperplane-ordered substitutions) against the oracle's sequential one (orc_sip_precond), on
the same seeded inputs, in FP64 and FP32, and solves with it."""
import numpy as np
import pytest

import oracle
import paper_1901_08269_amd as cps
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "sphere_stretched":        # (40, 40, 40), stretched, one sphere
        return W.sphere_sin(38, beta=1.4, r=0.27, c=(0.52, 0.47, 0.5))
    if name == "two_bodies_aniso":        # (70, 41, 29): unequal sides, a sphere and an ellipsoid
        x, y, z = W.tanh_grid(70, 1.5), W.tanh_grid(41, 1.0), W.uniform_grid(29)
        bodies = [W.Sphere((0.33, 0.45, 0.5), 0.17),
                  W.Ellipsoid((0.7, 0.55, 0.48), (0.16, 0.1, 0.2),
                              W._random_rotation(np.random.Generator(np.random.PCG64(5))))]
        return W.polynomial_case(0, bodies, rng_seed=9, grids=(x, y, z))
    if name == "wide_ragged":             # (283, 30, 21): rows longer than one thread block's span of j
        x, y, z = W.tanh_grid(283, 1.3), W.tanh_grid(30, 0.9), W.uniform_grid(21)
        return W.polynomial_case(0, [W.Sphere((0.3, 0.5, 0.5), 0.2)], rng_seed=21, grids=(x, y, z))
    if name == "interior":                # the fluid inside an ellipsoid, sinh-clustered y and z
        return W.interior_exp(42)
    raise KeyError(name)


CASES = ["sphere_stretched", "two_bodies_aniso", "wide_ragged", "interior"]


@pytest.mark.parametrize("alpha", [0.0, 0.9])
@pytest.mark.parametrize("name", CASES)
def test_sip_apply_matches_oracle(name, alpha):
    w = _case(name)
    print(f"[case] sip {name} alpha={alpha} shape {w.phi.shape}", flush=True)
    P = oracle.Problem.from_workload(w)
    t = P.types()
    unk = (t == 1) | (t == 2)
    rng = np.random.Generator(np.random.PCG64(3))
    rho = rng.standard_normal(P.shape) * unk
    F = P.sip_factors(alpha)
    for iters in (1, 3, 8):
        ref = P.precond_sip(rho, iters, factors=F)
        S = cps.Solver.from_workload(w, precond="sip", sip_iters=iters, sip_alpha=alpha)
        scale = np.max(np.abs(ref))
        for prec, bar in (("fp64", 1e-11), ("fp32", 2e-5)):
            got = S.precond(rho, precision=prec).cpu().numpy()
            err = np.max(np.abs(got - ref)) / scale
            print(f"  iters {iters} {prec}: max rel {err:.2e}")
            assert err <= bar, (iters, prec, err)
            assert np.all(got[~unk] == 0.0)
        S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_with_sip_matches_oracle(precision):
    w = _case("two_bodies_aniso")
    print(f"[case] sip solve two_bodies_aniso {precision}", flush=True)
    P = oracle.Problem.from_workload(w)
    u_ref, _ = P.solve(1e-13)
    t = P.types()
    fl = (t == 1) | (t == 2)
    S = cps.Solver.from_workload(w, precision=precision, precond="sip")
    u, st = S.solve(1e-12)
    assert st["rel_residual"] <= 1e-12 and st["rel_residual_jacobi"] <= 1e-12
    u = u.cpu().numpy()
    rel = np.max(np.abs(u - u_ref)[fl]) / np.max(np.abs(u_ref[fl]))
    print(f"{st['iters']} iterations, max rel. difference vs oracle {rel:.2e}")
    assert rel <= 1e-9
    assert np.all(u[t == 3] == 0.0)


def test_sip_options_validated():
    w = _case("sphere_stretched")
    for kw in ({"sip_iters": 0}, {"sip_iters": 65}, {"sip_alpha": -0.1}, {"sip_alpha": 1.5}):
        with pytest.raises(cps.CpsError):
            cps.Solver.from_workload(w, precond="sip", **kw)
