"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle on the same seeded
inputs -- setup tables, the B and preconditioner applies in FP64 and FP32, full solves in
plain FP64 and in mixed precision, edge cases and the full-size workloads on sampled nodes."""
import os

import numpy as np
import pytest

import oracle
import paper_1901_08269_amd as cps
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _box(x, y, z, lo, hi):
    Z, Y, X = W.mesh(x, y, z)
    d = [np.abs(c - 0.5 * (l + h)) - 0.5 * (h - l) for c, l, h in zip((X, Y, Z), lo, hi)]
    return np.broadcast_to(np.maximum(np.maximum(d[0], d[1]), d[2]), (len(z), len(y), len(x))).copy()


def _case(name):
    """Seeded parity cases: several 64x4 tiles with ragged tails, bodies of each kind."""
    if name == "nobody_ragged":
        rng = np.random.Generator(np.random.PCG64(1))
        x, y, z = W.random_grid(72, rng), W.tanh_grid(23, 1.2), W.tanh_grid(13, 0.8)
        w = W.polynomial_case(0, [], rng_seed=3, grids=(x, y, z))
        return w.x, w.y, w.z, w.phi, w.g, w.f, w.u_exact
    if name == "sphere_stretched":
        w = W.sphere_sin(38, beta=1.4, r=0.27, c=(0.52, 0.47, 0.5))
        return w.x, w.y, w.z, w.phi, w.g, w.f, w.u_exact
    if name == "two_bodies_aniso":
        x, y, z = W.tanh_grid(70, 1.5), W.tanh_grid(41, 1.0), W.uniform_grid(29)
        bodies = [W.Sphere((0.33, 0.45, 0.5), 0.17),
                  W.Ellipsoid((0.7, 0.55, 0.48), (0.16, 0.1, 0.2),
                              W._random_rotation(np.random.Generator(np.random.PCG64(5))))]
        w = W.polynomial_case(0, bodies, rng_seed=9, grids=(x, y, z))
        return w.x, w.y, w.z, w.phi, w.g, w.f, w.u_exact
    if name == "plates_fsf_sfs":
        x = W.uniform_grid(26)
        h = x[1] - x[0]
        phi = np.minimum(_box(x, x, x, (x[8] - 0.3 * h, 0.3, 0.3), (x[8] + 0.35 * h, 0.7, 0.7)),
                         _box(x, x, x, (x[10] - 0.4 * h, 0.3, 0.3), (x[12] + 0.3 * h, 0.7, 0.7)))
        phi = np.minimum(phi, _box(x, x, x, (0.3, x[1] + 0.5 * h, 0.3), (0.7, x[2] + 0.2 * h, 0.7)))
        Z, Y, X = W.mesh(x, x, x)
        u = np.broadcast_to(1 + X * X - 0.5 * Y * Y + 0.3 * Z * Z + 0.2 * X * Y, phi.shape).copy()
        return x, x, x, phi, u, np.full(phi.shape, 1.6), u
    if name == "near_coincident":
        x = W.uniform_grid(30)
        h = x[1] - x[0]
        w = W.polynomial_case(0, [], rng_seed=4, grids=(x, x, x))
        phi = _box(x, x, x, (0.3, x[11] + 1e-6 * h, 0.3), (0.7, x[15] + 0.5 * h, 0.7))
        return x, x, x, phi, w.g, w.f, w.u_exact
    if name == "wide_rows":
        # 298 interior nodes per x-row: the vectorised sweeps run two row segments (256 + 42)
        # and read the segment-edge neighbours from memory
        x, y, z = W.tanh_grid(300, 1.1), W.uniform_grid(14), W.uniform_grid(11)
        w = W.polynomial_case(0, [W.Sphere((0.78, 0.5, 0.47), 0.22)], rng_seed=11, grids=(x, y, z))
        return w.x, w.y, w.z, w.phi, w.g, w.f, w.u_exact
    if name == "interior":
        # the fluid region inside an ellipsoid, walls outside it (Problem 4's setting), on the
        # sinh grids of Eqs. p4_y / p4_z
        w = W.interior_exp(42)
        return w.x, w.y, w.z, w.phi, w.g, w.f, w.u_exact
    raise KeyError(name)


CASES = ["nobody_ragged", "sphere_stretched", "two_bodies_aniso", "plates_fsf_sfs", "near_coincident", "wide_rows",
         "interior"]


def _both(name, **kw):
    """The oracle's problem and the library's, the latter with the oracle's (Chebyshev)
    inner solver unless `precond` says otherwise."""
    x, y, z, phi, g, f, ue = _case(name)
    print(f"[case] {name} shape {phi.shape}", flush=True)
    P = oracle.Problem(x, y, z, phi, g, f)
    kw.setdefault("precond", "chebyshev")
    S = cps.Solver(x, y, z, phi, g, f, **kw)
    return P, S, ue


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_setup_tables(name):
    P, S, _ = _both(name)
    b_gpu, t_gpu = S.rhs_and_types()
    assert np.array_equal(_np(t_gpu), P.types())                       # node types: bit-exact
    oi, gi = P.info(), S.info()
    assert (gi["n_unknown"], gi["n_irregular"], gi["n_solid"]) == (oi["n_unknown"], oi["n_irregular"], oi["n_solid"])
    assert gi["fallback_lines"] == oi["fallback_lines"]
    node, ptr, col, val, krow = S.irregular()
    assert np.array_equal(node, P.irregular_nodes())                   # ordered irregular list
    rtol = 1e-8 if name == "near_coincident" else 1e-11
    for r, e in enumerate(node):
        oc, ov = P.row(e)
        c, v = col[ptr[r]:ptr[r + 1]], val[ptr[r]:ptr[r + 1]]
        order = np.argsort(c)
        assert np.array_equal(c[order], oc), (r, e)
        scale = np.max(np.abs(ov))
        assert np.max(np.abs(v[order] - ov)) <= rtol * scale, (r, e)
        ko = P.krow(e)
        assert np.max(np.abs(krow[r] - ko)) <= rtol * np.max(np.abs(ko)), (r, e)
    b = P.rhs()
    assert np.max(np.abs(_np(b_gpu) - b)) <= rtol * np.max(np.abs(b))


def _random_field(P, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(P.shape)
    return x


def _rounding_scale(P, x, grids):
    """Per-row magnitude that bounds the rounding of either evaluation order of B x:
    regular rows, sum_{p,q,r} (|R_x||L_y||L_z| + |L_x||R_y||L_z| + |L_x||L_y||R_z|) |x|
    (the three tensor terms of Eq. As_qs separately); irregular rows, sum_j |B_ij| |x_j|."""
    t = P.types()
    unk = (t == 1) | (t == 2)
    ax = np.where(unk, np.abs(x), 0.0)
    tabs = []
    for d, c in enumerate(grids):
        a, cc, ar, br, cr = (np.abs(v) for v in oracle.compact_coef(c))
        tabs.append(((a, np.ones_like(a), cc), (ar, br, cr)))

    def filt(v, d, w):
        axis = 2 - d                       # arrays are [z, y, x]
        shape = [1, 1, 1]
        shape[axis] = -1
        out = np.zeros_like(v)
        sl = [slice(None)] * 3
        for k, off in enumerate((-1, 0, 1)):
            src = np.roll(v, -off, axis=axis)
            out += w[k].reshape(shape) * src
        return out

    total = np.zeros_like(ax)
    for rdir in range(3):
        v = ax
        for d in range(3):
            v = filt(v, d, tabs[d][1] if d == rdir else tabs[d][0])
        total += v
    B, unk_idx = P.csr()
    irr = np.zeros(P.shape).ravel()
    irr[unk_idx] = abs(B) @ np.abs(x.ravel()[unk_idx])
    irr = irr.reshape(P.shape)
    return np.where(t == 2, irr, total)


@pytest.mark.parametrize("name", CASES)
def test_apply_fp64_and_fp32(name):
    """|y_gpu - y_oracle| <= c eps (rounding scale) per row: the kernel sums the regular
    rows by sum factorisation, a different order than the oracle's 27-term sum."""
    P, S, _ = _both(name)
    x = _random_field(P, 11)
    y_ref = P.apply(x)
    scale = _rounding_scale(P, x, _case(name)[:3])
    t = P.types()
    # irregular rows also carry the coefficient differences allowed by test_setup_tables
    # (the IBI roots come from different root finders on the two sides)
    coef_tol = np.where(t == 2, 1e-8 if name == "near_coincident" else 1e-11, 0.0)
    y64 = _np(S.apply(x, "fp64"))
    err64 = np.abs(y64 - y_ref)
    ratio64 = np.max(err64 / np.maximum(scale, 1e-300))
    print(f"fp64 max error / (eps * scale) = {ratio64 / 2.0 ** -52:.2f}, regular rows "
          f"{np.max((err64 / np.maximum(scale, 1e-300))[t == 1]) / 2.0 ** -52:.2f}")
    assert np.all(err64 <= (32 * 2.0 ** -52 + coef_tol) * scale)
    y32 = _np(S.apply(x, "fp32"))
    ratio32 = np.max(np.abs(y32 - y_ref) / np.maximum(scale, 1e-300))
    print(f"fp32 max error / (eps32 * scale) = {ratio32 / 2.0 ** -23:.2f}")
    assert ratio32 <= 32 * 2.0 ** -23


@pytest.mark.parametrize("name", CASES)
def test_precond_fp64_and_fp32(name):
    P, S, _ = _both(name)
    rho = _random_field(P, 12)
    # default interval policy on both sides (lo = hi / (4 m^2)), and one explicit interval
    for m, lo in ((1, None), (8, 0.03), (24, None)):
        S2 = cps.Solver(*_case(name)[:6], inner_iters=m, lam_lo=lo, precond="chebyshev")
        ref = P.precond(rho, iters=m, lo=lo)
        scale = np.max(np.abs(ref))
        got = _np(S2.precond(rho, "fp64"))
        assert np.max(np.abs(got - ref)) <= 1e-11 * scale, m
        got32 = _np(S2.precond(rho, "fp32"))
        assert np.max(np.abs(got32 - ref)) <= 1e-5 * scale, m


@pytest.mark.parametrize("name", CASES)
def test_solve_fp64_matches_oracle(name):
    P, S, ue = _both(name)
    t = P.types()
    fl = (t == 1) | (t == 2)
    # Ill-conditioned cases converge further before the 1e-10 comparison: an oracle solve of
    # the near-coincident case at 1e-13 differs from one at 1e-15 by ~5e-10, one of the
    # wide-row case (many fallback lines, an IBI at 9e-4 h) at 1e-12 by 8.9e-11.
    tol = 1e-14 if name in ("near_coincident", "wide_rows") else 1e-12
    u_ref, st_ref = P.solve(tol / 10)
    u, st = S.solve(tol)
    u = _np(u)
    assert st["rel_residual"] <= tol and st["rel_residual_jacobi"] <= tol
    rel = np.max(np.abs(u - u_ref)[fl]) / np.max(np.abs(u_ref[fl]))
    assert rel <= 1e-10, rel
    assert np.all(u[t == 3] == 0.0)                 # exactly zero inside bodies
    assert np.array_equal(u[t == 0], _case(name)[4][t == 0])   # g on the walls
    assert abs(st["iters"] - st_ref["iters"]) <= max(3, st_ref["iters"] // 4)


@pytest.mark.parametrize("name", ["sphere_stretched", "two_bodies_aniso", "plates_fsf_sfs"])
def test_solve_mixed_matches_oracle(name):
    P, S, ue = _both(name, precision="mixed")
    t = P.types()
    fl = (t == 1) | (t == 2)
    u_ref, _ = P.solve(1e-13)
    u, st = S.solve(1e-11)
    u = _np(u)
    assert st["refine_steps"] >= 2 and st["iters_fp32"] == st["iters"]
    assert st["rel_residual"] <= 1e-11 and st["rel_residual_jacobi"] <= 1e-11
    rel = np.max(np.abs(u - u_ref)[fl]) / np.max(np.abs(u_ref[fl]))
    assert rel <= 1e-9, rel


def test_residual_matches_oracle():
    P, S, _ = _both("two_bodies_aniso")
    x = _random_field(P, 5)
    r_ref, rel_ref = P.residual(x)
    r, rel, rel_j = S.residual(x)
    assert np.max(np.abs(_np(r) - r_ref)) <= 1e-12 * np.max(np.abs(r_ref))
    assert abs(rel - rel_ref) <= 1e-12 * rel_ref


def test_determinism_bitwise():
    _, S, _ = _both("sphere_stretched")
    u1, s1 = S.solve(1e-10)
    u1 = _np(u1).copy()
    u2, s2 = S.solve(1e-10)
    assert np.array_equal(u1, _np(u2)) and s1["iters"] == s2["iters"]


def test_warm_start_exact_and_nan():
    P, S, _ = _both("sphere_stretched")
    u_ref, _ = P.solve(1e-13)
    u, st = S.solve(1e-10, u0=u_ref)
    assert st["iters"] == 0
    bad = u_ref.copy()
    bad[5, 5, 5] = np.nan
    u, st = S.solve(1e-10, u0=bad)
    assert st["status"] == 0 and np.all(np.isfinite(_np(u)))


def test_warm_start_scaled_never_worse():
    """A warm start whose residual exceeds ||b|| is scaled by argmin ||b - alpha B u0||: an
    exact start keeps alpha = 1, a start whose residual far exceeds ||b|| is scaled down and
    costs at most as many iterations as a zero start (plus the rounding of a slightly
    different start)."""
    P, S, _ = _both("sphere_stretched")
    t = P.types()
    u_ref, _ = P.solve(1e-13)
    u, st = S.solve(1e-10, u0=u_ref)
    assert st["iters"] == 0 and abs(st["warm_alpha"] - 1.0) < 1e-9
    _, st0 = S.solve(1e-10)
    assert st0["warm_alpha"] == 0.0
    rng = np.random.Generator(np.random.PCG64(3))
    noisy = u_ref + 1e3 * rng.standard_normal(u_ref.shape) * ((t == 1) | (t == 2))
    u, st = S.solve(1e-10, u0=noisy)
    assert 0.0 <= st["warm_alpha"] < 1e-2
    assert st["iters"] <= st0["iters"] + 2
    assert st["rel_residual"] <= 1e-10


def test_max_iters_exit():
    x, y, z, phi, g, f, _ = _case("sphere_stretched")
    S = cps.Solver(x, y, z, phi, g, f, max_iters=2)
    u, st = S.solve(1e-14, check=False)
    assert st["status"] == -6 and st["iters"] == 2
    assert np.all(np.isfinite(_np(u)))


def test_invalid_geometry_rejected():
    x = W.uniform_grid(12)
    phi = np.ones((12, 12, 12))
    phi[0, 4, 4] = -1.0
    with pytest.raises(cps.CpsError) as e:
        cps.Solver(x, x, x, phi, phi, phi)
    assert e.value.code == -2
    phi = np.ones((12, 12, 12))
    f = phi.copy()
    f[3, 3, 3] = np.inf
    with pytest.raises(cps.CpsError) as e:
        cps.Solver(x, x, x, phi, phi, f)
    assert e.value.code == -1


def test_smallest_grid():
    # one interior node, no body
    x = W.uniform_grid(3)
    Z, Y, X = W.mesh(x, x, x)
    g = np.broadcast_to(X * X + Y, (3, 3, 3)).copy()
    f = np.full((3, 3, 3), 2.0)
    P = oracle.Problem(x, x, x, np.ones_like(g), g, f)
    S = cps.Solver(x, x, x, np.ones_like(g), g, f)
    u_ref, _ = P.solve(1e-13)
    u, st = S.solve(1e-12)
    assert abs(_np(u)[1, 1, 1] - u_ref[1, 1, 1]) <= 1e-12 * abs(u_ref[1, 1, 1])


def test_zero_rhs_and_no_unknowns():
    """Degenerate problems: f = g = 0 gives b = 0, which a zero start already solves (no
    iteration, no division by ||b|| = 0, also with a nonzero warm start, which the
    residual-based scaling sends to zero); a body filling the whole interior leaves no
    unknown at all, and the output is g on the walls and 0 inside."""
    x = W.uniform_grid(10)
    Z, Y, X = W.mesh(x, x, x)
    phi = np.ones((10, 10, 10))
    zero = np.zeros_like(phi)
    for prec in ("fp64", "mixed"):
        S = cps.Solver(x, x, x, phi, zero, zero, precision=prec)
        u, st = S.solve(1e-10)
        assert st["status"] == 0 and st["iters"] == 0 and np.all(_np(u) == 0.0)
        u, st = S.solve(1e-10, u0=np.ones_like(phi))
        assert st["status"] == 0 and np.all(_np(u) == 0.0)
        S.close()
    phi2 = -np.ones_like(phi)
    wall = np.zeros(phi.shape, dtype=bool)
    wall[0], wall[-1], wall[:, 0], wall[:, -1], wall[:, :, 0], wall[:, :, -1] = True, True, True, True, True, True
    phi2[wall] = 1.0
    g = np.broadcast_to(1.0 + X + 2.0 * Y, phi.shape).copy()
    S = cps.Solver(x, x, x, phi2, g, np.ones_like(phi), precision="mixed")
    u, st = S.solve(1e-10)
    assert st["status"] == 0 and st["n_unknowns"] == 0 and st["iters"] == 0
    uu = _np(u)
    assert np.array_equal(uu[wall], g[wall]) and np.all(uu[~wall] == 0.0)


# ----------------------------------------------------------------------------------------
# full-size workloads against stored oracle samples
# ----------------------------------------------------------------------------------------
def _samples(fname):
    path = os.path.join(GOLD, fname)
    if not os.path.exists(path):
        pytest.skip(f"{fname} not generated")
    data = np.loadtxt(path, comments="#")
    umax = None
    for line in open(path):
        if line.startswith("# max_abs_u_fluid"):
            umax = float(line.split()[-1])
    return data[:, 0].astype(np.int64), data[:, 1], umax


def test_sphere_exp_128_fp64_vs_oracle_samples():
    nodes, vals, umax = _samples("oracle_sphere_exp_128.txt")
    w = W.sphere_exp(128)
    print("[case] sphere_exp 128 FP64", flush=True)
    S = cps.Solver.from_workload(w)
    u, st = S.solve(1e-12)
    got = _np(u).ravel()[nodes]
    assert np.max(np.abs(got - vals)) / umax <= 1e-10
    assert st["rel_residual"] <= 1e-12


def test_spheres8_256_mixed_vs_oracle_samples():
    """256^3, 8 spheres.  At tol 1e-10 the residual bound holds but the iteration error
    (~1e-7) exceeds 1e-9 at this size: a residual of 1e-12 still leaves ~1e-9 of it.  At
    tol 1e-13 both the mixed and the plain FP64 solution match the FP64 oracle (solved to
    1e-13, Jacobi-weighted residual 6e-14) to <= 1e-9 relative max-norm on the samples."""
    nodes, vals, umax = _samples("oracle_spheres8_256.txt")
    w = W.spheres8(256)
    print("[case] spheres8 256 mixed", flush=True)
    S = cps.Solver.from_workload(w, precision="mixed")
    u, st = S.solve(1e-10)
    assert st["rel_residual"] <= 1e-10 and st["rel_residual_jacobi"] <= 1e-10
    assert st["fallback_lines"] == 0
    u, st = S.solve(1e-13)
    assert st["rel_residual"] <= 1e-13 and st["rel_residual_jacobi"] <= 1e-13
    got = _np(u).ravel()[nodes]
    rel = np.max(np.abs(got - vals)) / umax
    print(f"mixed: max rel. difference vs oracle samples: {rel:.2e}")
    assert rel <= 1e-9
    S.close()
    print("[case] spheres8 256 fp64", flush=True)
    S = cps.Solver.from_workload(w, precision="fp64")
    u, st = S.solve(1e-13)
    assert st["rel_residual"] <= 1e-13 and st["rel_residual_jacobi"] <= 1e-13
    rel = np.max(np.abs(_np(u).ravel()[nodes] - vals)) / umax
    print(f"fp64: max rel. difference vs oracle samples: {rel:.2e}")
    assert rel <= 1e-9


def test_star_fourier_128_vs_oracle_samples():
    """128^3, star-shaped body, random Fourier f, g = 0 (the learned warm start's family, at
    its full size): the plain FP64 and the mixed solution at tol 1e-13 against the FP64
    oracle solved to 1e-13, on the stored samples (every 7th irregular node plus uniformly
    drawn fluid nodes).  The star's thin arms make short marches (fallback lines), which
    both sides count alike."""
    nodes, vals, umax = _samples("oracle_star_fourier_128.txt")
    fb = None
    for line in open(os.path.join(GOLD, "oracle_star_fourier_128.txt")):
        if line.startswith("# info"):
            fb = int(line.split("'fallback_lines': ")[1].split(",")[0])
    w = W.star_fourier(128)
    for prec in ("fp64", "mixed"):
        print(f"[case] star_fourier 128 {prec}", flush=True)
        S = cps.Solver.from_workload(w, precision=prec)
        u, st = S.solve(1e-13)
        assert st["rel_residual"] <= 1e-13 and st["rel_residual_jacobi"] <= 1e-13
        assert st["fallback_lines"] == fb
        rel = np.max(np.abs(_np(u).ravel()[nodes] - vals)) / umax
        print(f"{prec}: max rel. difference vs oracle samples: {rel:.2e}")
        assert rel <= 1e-9
        S.close()


def _subbox(x, body, margin):
    """Index range [lo, hi] per axis covering the body's bounding sphere plus `margin` cells."""
    lo, hi = [], []
    for d in range(3):
        a = int(np.searchsorted(x, body.c[d] - body.bound)) - margin
        b = int(np.searchsorted(x, body.c[d] + body.bound)) + margin
        lo.append(max(a, 0))
        hi.append(min(b, len(x) - 1))
    return lo, hi


@pytest.mark.parametrize("precond", ["chebyshev", "multigrid"])
def test_bodies16_512_rows_vs_oracle(precond):
    """512^3, 8 spheres + 8 rotated ellipsoids, Fourier f with 2445 modes, g = 0: the scale
    configuration, too large for an oracle solve.  The GPU's mixed solution to 1e-10 is
    checked against the oracle's own system, row by row: around two bodies the oracle builds
    the problem on a sub-box of the grid (its rows at least 6 cells inside the sub-box only
    see nodes of the sub-box, and every row of the discretisation is local), and at every
    irregular row and 2000 regular rows there it forms b_i - (B u)_i with the GPU solution.
    Relative to the row's scale |b_i| + sum_j |B_ij u_j| these residuals must stay at the
    solve's tolerance (1e-10; measured up to 2e-12), which a wrong coefficient anywhere in a
    sampled row would exceed.  One sub-box around a sphere, one around an ellipsoid."""
    import torch
    x, bodies, phi, g, f = W.bodies16_fourier_torch(512)
    n = len(x)
    print(f"[case] bodies16_fourier 512 mixed, {precond}", flush=True)
    S = cps.Solver(x, x, x, phi, g, f, precision="mixed", precond=precond)
    u, st = S.solve(1e-10)
    assert st["rel_residual"] <= 1e-10 and st["rel_residual_jacobi"] <= 1e-10
    assert st["fallback_lines"] == 0
    S.close()
    uflat = u.reshape(-1)
    rng = np.random.Generator(np.random.PCG64(7))
    done = set()
    for b in bodies:
        kind = type(b).__name__
        if kind in done:
            continue   # one sphere and one ellipsoid
        lo, hi = _subbox(x, b, 8)
        sl = (slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
        ph = phi[sl].cpu().numpy()
        faces = [ph[0], ph[-1], ph[:, 0], ph[:, -1], ph[:, :, 0], ph[:, :, -1]]
        if min(float(a.min()) for a in faces) <= 0.0:
            continue   # another body crosses the sub-box boundary
        xs, ys, zs = x[lo[0]:hi[0] + 1], x[lo[1]:hi[1] + 1], x[lo[2]:hi[2] + 1]
        P = oracle.Problem(xs, ys, zs, ph, g[sl].cpu().numpy(), f[sl].cpu().numpy())
        t = P.types()
        nz_, ny_, nx_ = t.shape
        K, J, I = np.meshgrid(np.arange(nz_), np.arange(ny_), np.arange(nx_), indexing="ij")
        inner = (I >= 6) & (I <= nx_ - 7) & (J >= 6) & (J <= ny_ - 7) & (K >= 6) & (K <= nz_ - 7)
        irr = np.nonzero((t == 2) & inner)
        reg = np.nonzero((t == 1) & inner)
        pick = rng.choice(len(reg[0]), size=min(2000, len(reg[0])), replace=False)
        rows = [(k, j, i) for k, j, i in zip(*irr)] + [(reg[0][q], reg[1][q], reg[2][q]) for q in pick]
        bsub = P.rhs()
        cols_all, vals_all, owner = [], [], []
        bvals = np.empty(len(rows))
        for r, (k, j, i) in enumerate(rows):
            e = int(i + nx_ * (j + ny_ * k))
            c, v = P.row(e)
            cols_all.append(c)
            vals_all.append(v)
            owner.append(np.full(len(c), r))
            bvals[r] = bsub[k, j, i]
        cols = np.concatenate(cols_all)
        ci, cj, ck = cols % nx_, (cols // nx_) % ny_, cols // (nx_ * ny_)
        full = (ci + lo[0]) + n * ((cj + lo[1]) + n * (ck + lo[2]))
        uval = uflat[torch.as_tensor(full, device=uflat.device)].cpu().numpy()
        vals = np.concatenate(vals_all)
        own = np.concatenate(owner)
        bu = np.bincount(own, weights=vals * uval, minlength=len(rows))
        scale = np.abs(bvals) + np.bincount(own, weights=np.abs(vals * uval), minlength=len(rows))
        ratio = np.max(np.abs(bvals - bu) / scale)
        print(f"body {type(b).__name__} box {[h - l + 1 for l, h in zip(lo, hi)]}: {len(irr[0])} irregular "
              f"+ {len(pick)} regular rows, max |b - Bu| / scale = {ratio:.2e}")
        assert len(irr[0]) > 100
        assert ratio <= 1e-10
        done.add(kind)
    assert done == {"Sphere", "Ellipsoid"}
