"""Pins of the oracle's 1D coefficients (Eqs. app_xxx and 2ndorder_coef) and of the
one-sided modified operators (Eqs. mod1-mod4 with their systems mat1-mat4 and M;
Sec. 2.3 Eqs. mod2_case2 / mod2_case22)."""
import numpy as np
import pytest

import oracle
from paper_1901_08269_amd import workloads as W


def _grids():
    rng = np.random.Generator(np.random.PCG64(3))
    return [W.uniform_grid(17), W.tanh_grid(33, 2.0), W.random_grid(25, rng, 0.45)]


def test_compact_uniform_limit():
    # uniform spacing h: (a, b, c) = (1/10, 1, 1/10), (ar, br, cr) = (6/5, -12/5, 6/5) / h^2
    x = W.uniform_grid(21)
    h = x[1] - x[0]
    a, c, ar, br, cr = oracle.compact_coef(x)
    s = slice(1, -1)
    np.testing.assert_allclose(a[s], 0.1, rtol=1e-13)
    np.testing.assert_allclose(c[s], 0.1, rtol=1e-13)
    np.testing.assert_allclose(ar[s] * h * h, 1.2, rtol=1e-12)
    np.testing.assert_allclose(br[s] * h * h, -2.4, rtol=1e-12)
    np.testing.assert_allclose(cr[s] * h * h, 1.2, rtol=1e-12)


@pytest.mark.parametrize("gi", range(3))
def test_compact_moment_identities(gi):
    x = _grids()[gi]
    a, c, ar, br, cr = oracle.compact_coef(x)
    i = np.arange(1, len(x) - 1)
    dxf, dxb = x[i + 1] - x[i], x[i] - x[i - 1]
    scale = np.abs(br[i])
    np.testing.assert_allclose((ar[i] + br[i] + cr[i]) / scale, 0, atol=1e-13)
    np.testing.assert_allclose((-ar[i] * dxb + cr[i] * dxf) / (scale * dxf), 0, atol=1e-13)
    np.testing.assert_allclose(0.5 * (ar[i] * dxb ** 2 + cr[i] * dxf ** 2), a[i] + 1.0 + c[i], rtol=1e-12)


@pytest.mark.parametrize("gi", range(3))
def test_compact_polynomial_exactness(gi):
    # a u''_{i-1} + u''_i + c u''_{i+1} = ar u_{i-1} + br u_i + cr u_{i+1} for degree <= 4
    x = _grids()[gi]
    a, c, ar, br, cr = oracle.compact_coef(x)
    i = np.arange(1, len(x) - 1)
    for m in range(0, 6):
        xc = x - 0.37  # shifted monomials keep the check away from symmetric special cases
        u = xc ** m
        upp = m * (m - 1) * xc ** (m - 2) if m >= 2 else 0 * xc
        lhs = a[i] * upp[i - 1] + upp[i] + c[i] * upp[i + 1]
        rhs = ar[i] * u[i - 1] + br[i] * u[i] + cr[i] * u[i + 1]
        err = np.max(np.abs(lhs - rhs)) / max(1.0, np.max(np.abs(br[i] * u[i])))
        if m <= 4:
            assert err < 1e-11, (m, err)
        elif gi != 0:
            assert err > 1e-8, "degree 5 must not be reproduced on a nonuniform grid"


@pytest.mark.parametrize("gi", range(3))
def test_second_order_coefficients(gi):
    x = _grids()[gi]
    a, b, c = oracle.second_coef(x)
    i = np.arange(1, len(x) - 1)
    for m in range(0, 3):
        u = (x - 0.2) ** m
        upp = m * (m - 1) * (x - 0.2) ** (m - 2) if m >= 2 else 0 * x
        np.testing.assert_allclose(a[i] * u[i - 1] + b[i] * u[i] + c[i] * u[i + 1], upp[i],
                                   atol=1e-9 * np.max(np.abs(b)))


# ----------------------------------------------------------------------------------------
# one-sided operators: the printed Taylor systems of Sec. 2.2
# ----------------------------------------------------------------------------------------
def _M(h):
    """Eq. (M): first column (1,0,...,0), then columns (1, h, h^2, ..., h^5) per offset."""
    M = np.zeros((6, 6))
    M[0, :] = 1.0
    for col, hc in enumerate(h, start=1):
        for row in range(1, 6):
            M[row, col] = hc ** row
    return M


def _line(seed, n=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    return W.random_grid(n, rng, 0.4)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mat1(seed):
    # Eqs. mod1_top/mod1/mat1: run {i-1, i} with L weights (a, b=1), solid at i+1, extras
    # i-2, i-3, i-4, IBI in (x_i, x_{i+1}); unknowns [br, ar, psi1, psi2, psi3, psi_b].
    x = _line(seed)
    i = 6
    a, c, ar, br, cr = oracle.compact_coef(x)
    xb = x[i] + 0.37 * (x[i + 1] - x[i])
    h = [x[i - 1] - x[i], x[i - 2] - x[i], x[i - 3] - x[i], x[i - 4] - x[i], xb - x[i]]
    h0 = h[0]
    rhs = np.array([0, 0, 2 * (a[i] + 1.0), 6 * h0 * a[i], 12 * h0 ** 2 * a[i], 20 * h0 ** 3 * a[i]])
    paper = np.linalg.solve(_M(h), rhs)
    pts = [x[i], x[i - 1], x[i - 2], x[i - 3], x[i - 4], xb]
    w = oracle.onesided_weights(pts, [x[i - 1], x[i]], [a[i], 1.0], tref=x[i])
    np.testing.assert_allclose(w, paper, rtol=1e-8, atol=1e-10 * np.max(np.abs(paper)))


@pytest.mark.parametrize("seed", [4, 5])
def test_mat2(seed):
    # Eqs. mod2_top/mod2/mat2: run {j-1} with weight a, extras j-2..j-5, IBI in (y_{j-1}, y_j);
    # Taylor about y_{j-1}; unknowns [ar, beta1..beta4, beta_b].
    y = _line(seed, 14)
    j = 8
    a, c, ar, br, cr = oracle.compact_coef(y)
    yb = y[j - 1] + 0.61 * (y[j] - y[j - 1])
    h = [y[j - 2] - y[j - 1], y[j - 3] - y[j - 1], y[j - 4] - y[j - 1], y[j - 5] - y[j - 1], yb - y[j - 1]]
    rhs = np.array([0, 0, 2 * a[j], 0, 0, 0])
    paper = np.linalg.solve(_M(h), rhs)
    pts = [y[j - 1], y[j - 2], y[j - 3], y[j - 4], y[j - 5], yb]
    w = oracle.onesided_weights(pts, [y[j - 1]], [a[j]], tref=y[j - 1])
    np.testing.assert_allclose(w, paper, rtol=1e-8, atol=1e-10 * np.max(np.abs(paper)))


@pytest.mark.parametrize("seed", [6, 7])
def test_mat3(seed):
    # Eqs. mod3_top/mod3/mat3: run {k, k+1} with weights (b=1, c), solid at k-1, IBI in
    # (z_{k-1}, z_k), extras k+2..k+4; Taylor about z_k; unknowns [br, cr, th1, th2, th3, th_b].
    z = _line(seed)
    k = 4
    a, c, ar, br, cr = oracle.compact_coef(z)
    zb = z[k] - 0.29 * (z[k] - z[k - 1])
    h = [z[k + 1] - z[k], z[k + 2] - z[k], z[k + 3] - z[k], z[k + 4] - z[k], zb - z[k]]
    h0 = h[0]
    rhs = np.array([0, 0, 2 * (1.0 + c[k]), 6 * h0 * c[k], 12 * h0 ** 2 * c[k], 20 * h0 ** 3 * c[k]])
    paper = np.linalg.solve(_M(h), rhs)
    pts = [z[k], z[k + 1], z[k + 2], z[k + 3], z[k + 4], zb]
    w = oracle.onesided_weights(pts, [z[k], z[k + 1]], [1.0, c[k]], tref=z[k])
    np.testing.assert_allclose(w, paper, rtol=1e-8, atol=1e-10 * np.max(np.abs(paper)))


@pytest.mark.parametrize("seed", [8, 9])
def test_mat4(seed):
    # Eqs. mod4_top/mod4/mat4: run {k+1} with weight c, extras k+2..k+5, IBI in
    # (z_k, z_{k+1}); Taylor about z_{k+1}; unknowns [cr, th1..th4, th_b].
    z = _line(seed, 14)
    k = 3
    a, c, ar, br, cr = oracle.compact_coef(z)
    zb = z[k] + 0.12 * (z[k + 1] - z[k])
    h = [z[k + 2] - z[k + 1], z[k + 3] - z[k + 1], z[k + 4] - z[k + 1], z[k + 5] - z[k + 1], zb - z[k + 1]]
    rhs = np.array([0, 0, 2 * c[k], 0, 0, 0])
    paper = np.linalg.solve(_M(h), rhs)
    pts = [z[k + 1], z[k + 2], z[k + 3], z[k + 4], z[k + 5], zb]
    w = oracle.onesided_weights(pts, [z[k + 1]], [c[k]], tref=z[k + 1])
    np.testing.assert_allclose(w, paper, rtol=1e-8, atol=1e-10 * np.max(np.abs(paper)))


@pytest.mark.parametrize("npts,seed", [(5, 11), (6, 12), (3, 13)])
def test_onesided_exactness_degree(npts, seed):
    # the weights reproduce sum L[p] u''(x_p) for every polynomial of degree < |P| and not
    # for degree |P| (5 points: the F-S-F sides of Sec. 2.3; 3 points: S-F-S)
    x = _line(seed, 12)
    pts = list(x[2:2 + npts - 1]) + [x[2 + npts - 1] - 0.3 * (x[2 + npts - 1] - x[2 + npts - 2])]
    tr, Lw = [x[2]], [0.13]
    w = oracle.onesided_weights(pts, tr, Lw, tref=x[2])
    pts = np.array(pts)
    for m in range(npts + 1):
        lhs = np.dot(w, (pts - 0.4) ** m)
        rhs = Lw[0] * (m * (m - 1) * (tr[0] - 0.4) ** (m - 2) if m >= 2 else 0.0)
        scale = np.sum(np.abs(w) * np.abs(pts - 0.4) ** m) + 1.0
        if m < npts:
            assert abs(lhs - rhs) < 1e-10 * scale, (m, lhs, rhs)
        else:
            assert abs(lhs - rhs) > 1e-6 * scale, m
