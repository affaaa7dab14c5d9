"""Pins of the oracle's multigrid preconditioner for K (an inner solver for the K-preconditioned
BiCGSTAB of Sec. 3.3; the paper allows other inner solvers than the one it uses).

Each pin checks one part against a route that does not reuse the part: the transfer operators
against exact interpolation and the transpose definition, the smoother against the algebra of
Chebyshev iteration, and the whole cycle against a dense direct solve on a tiny grid."""
import numpy as np

import oracle
from oracle import mg
from paper_1901_08269_amd import workloads as W


def _sphere_problem(n, r=0.27):
    x = W.tanh_grid(n, 1.2)
    phi = W.union_level([W.Sphere((0.5, 0.47, 0.52), r)], x, x, x)
    return x, phi


def test_coarse_indices_keep_even_points_and_the_wall():
    assert list(mg.coarse_indices(9)) == [0, 2, 4, 6, 8]
    assert list(mg.coarse_indices(10)) == [0, 2, 4, 6, 8, 9]
    assert list(mg.coarse_indices(3)) == [0, 2]


def test_prolongation_exact_on_trilinear_fields():
    """Tensor-product linear interpolation in the physical coordinates reproduces any
    trilinear function of (x, y, z) exactly, on a stretched grid and an odd/even mix of sizes."""
    xs = (W.tanh_grid(13, 1.5), W.tanh_grid(12, 1.1), W.uniform_grid(10))
    idx = [mg.coarse_indices(len(c)) for c in xs]
    xc = [c[i] for c, i in zip(xs, idx)]
    ax = [mg.interp_1d(f, c, i) for f, c, i in zip(xs, xc, idx)]

    def field(x, y, z):
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return 0.7 - 1.3 * X + 2.1 * Y + 0.4 * Z + 0.9 * X * Y - 1.7 * Y * Z + 0.3 * X * Z + 2.5 * X * Y * Z

    fine = mg.prolong(field(*xc), ax)
    np.testing.assert_allclose(fine, field(*xs), rtol=0, atol=1e-13)


def test_restriction_is_normalised_transpose_of_prolongation():
    """R = D^-1 P^T with D the row sums of P^T: P is assembled column by column from prolong()
    of unit vectors (brute force), R applied through restrict()."""
    xs = (W.tanh_grid(7, 1.3), W.tanh_grid(6, 1.0), W.uniform_grid(5))
    idx = [mg.coarse_indices(len(c)) for c in xs]
    xc = [c[i] for c, i in zip(xs, idx)]
    ax = [mg.interp_1d(f, c, i) for f, c, i in zip(xs, xc, idx)]
    shape_f = (len(xs[2]), len(xs[1]), len(xs[0]))
    shape_c = (len(xc[2]), len(xc[1]), len(xc[0]))
    nc = int(np.prod(shape_c))
    P = np.zeros((int(np.prod(shape_f)), nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        P[:, j] = mg.prolong(e.reshape(shape_c), ax).ravel()
    rng = np.random.default_rng(5)
    r = rng.standard_normal(shape_f)
    expect = (P.T @ r.ravel()) / P.sum(axis=0)
    np.testing.assert_allclose(mg.restrict(r, ax, shape_c).ravel(), expect, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(mg.restrict(np.ones(shape_f), ax, shape_c), 1.0, rtol=1e-14)


def test_smoother_from_a_guess_is_guess_plus_correction():
    """Chebyshev iteration is affine in its start: from x0 it returns x0 plus the iterate
    from 0 for the residual rho - K x0 (same polynomial of diag(K)^-1 K)."""
    x, phi = _sphere_problem(18)
    P = oracle.Problem.k_only(x, x, x, phi)
    unk = np.isin(P.types(), (1, 2))
    rng = np.random.default_rng(1)
    rho = rng.standard_normal(phi.shape) * unk
    x0 = rng.standard_normal(phi.shape) * unk
    a = P.smooth(rho, x0, 5, 0.5, 2.0)
    b = x0 + P.smooth(rho - P.apply_K(x0), np.zeros_like(x0), 5, 0.5, 2.0)
    np.testing.assert_allclose(a[unk], b[unk], rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_k_only_levels_match_the_full_problem():
    """A level built from the level set alone has the full problem's node types and K rows."""
    x, phi = _sphere_problem(16)
    one = np.ones_like(phi)
    full = oracle.Problem(x, x, x, phi, one, one)
    konly = oracle.Problem.k_only(x, x, x, phi)
    np.testing.assert_array_equal(full.types(), konly.types())
    rng = np.random.default_rng(2)
    v = rng.standard_normal(phi.shape)
    np.testing.assert_allclose(konly.apply_K(v), full.apply_K(v), rtol=0, atol=0)


def _dense_K(P, unk):
    nodes = np.flatnonzero(unk.ravel())
    A = np.zeros((len(nodes), len(nodes)))
    for j, nd in enumerate(nodes):
        e = np.zeros(unk.size)
        e[nd] = 1.0
        A[:, j] = P.apply_K(e.reshape(unk.shape)).ravel()[nodes]
    return A, nodes


def test_vcycle_is_linear_and_converges_as_a_stationary_iteration():
    """M is a fixed linear map, and x <- x + M (rho - K x) contracts the error of the dense
    direct solution of K x = rho by a grid-independent factor (here < 0.6 per cycle over 8)."""
    x, phi = _sphere_problem(22)
    M = mg.Multigrid(x, x, x, phi, levels=3, min_points=5, coarse_interior=0)
    assert len(M.lv) == 3
    K0 = M.lv[0]["P"]
    unk = M.lv[0]["unk"].astype(bool)
    rng = np.random.default_rng(3)
    r1, r2 = rng.standard_normal(phi.shape) * unk, rng.standard_normal(phi.shape) * unk
    lhs = M.apply(2.0 * r1 - 0.5 * r2)
    rhs = 2.0 * M.apply(r1) - 0.5 * M.apply(r2)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())

    A, nodes = _dense_K(K0, unk)
    exact = np.zeros(phi.size)
    exact[nodes] = np.linalg.solve(A, r1.ravel()[nodes])
    exact = exact.reshape(phi.shape)
    xk = np.zeros_like(r1)
    errs = [np.abs(exact).max()]
    for _ in range(8):
        xk = xk + M.apply((r1 - K0.apply_K(xk)) * unk)
        errs.append(np.abs(xk - exact).max())
    rate = (errs[-1] / errs[0]) ** (1 / 8)
    assert rate < 0.6, errs
    assert np.all(np.diff(errs) < 0), errs


def test_vcycle_zero_outside_unknowns():
    x, phi = _sphere_problem(20)
    M = mg.Multigrid(x, x, x, phi, levels=2, min_points=5)
    rng = np.random.default_rng(4)
    out = M.apply(rng.standard_normal(phi.shape))
    unk = M.lv[0]["unk"].astype(bool)
    assert np.all(out[~unk] == 0.0)
    assert np.abs(out[unk]).max() > 0
