"""Pins for the paper's other workload forms (Sec. 4): the interior-clustering sinh grid map
(Eqs. p2_y, p2_s, p4_y, p4_z) and an interior problem (Problem 4, Eq. p4: the fluid region
inside a closed interface, the walls outside it)."""
import math

import numpy as np
import pytest

import oracle
from paper_1901_08269_amd import workloads as W


@pytest.mark.parametrize("beta,L,H,y0", [(3.0, 0.3, 0.6, -0.3), (2.0, 0.14, 0.5, 0.0), (4.0, 0.15, 0.3, 0.35)])
def test_sinh_grid_spans_the_domain_and_clusters_at_L(beta, L, H, y0):
    """With s of Eq. p2_s the map reaches y0 + H at eta = 1 (checked on the formula before the
    ends are set), passes y0 + L at eta = s, and is densest there."""
    n = 65
    y = W.sinh_grid(n, beta, L, H, y0)
    s = math.log((1 + (math.exp(beta) - 1) * L / H) / (1 + (math.exp(-beta) - 1) * L / H)) / (2 * beta)
    end = y0 + L * (1 + math.sinh(beta * (1 - s)) / math.sinh(beta * s))
    assert abs(end - (y0 + H)) < 1e-12
    assert y[0] == y0 and y[-1] == y0 + H
    h = np.diff(y)
    assert np.all(h > 0)
    q = int(np.argmin(h))
    assert y[q] - 1e-12 <= y0 + L <= y[q + 1] + 2 * h[q]
    # densest near y0 + L, coarsest at an end
    assert h[q] < 0.5 * max(h[0], h[-1])


def test_interior_problem_is_fourth_order():
    """Problem 4's solution u = exp(-10 r) on the p4 grids, solved inside an ellipsoid (a stand
    in for the figure-only pipe): the max-norm error falls at fourth order (measured 3.92 and
    4.05 between n = 26, 42, 74)."""
    errs, hs = [], []
    for n in (26, 42, 74):
        w = W.interior_exp(n)
        P = oracle.Problem.from_workload(w)
        u, st = P.solve(1e-12)
        t = P.types()
        fl = (t == 1) | (t == 2)
        assert fl.sum() > 0 and np.all(t[0] == 0)          # walls are in the body, kept as walls
        errs.append(np.max(np.abs(u - w.u_exact)[fl]))
        hs.append(1.0 / (n - 1))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(2)]
    assert min(orders) > 3.6, (errs, orders)
    assert errs[-1] < 2e-8


def test_walls_inside_a_body_need_solid_neighbours():
    """A wall node with phi <= 0 is accepted when its interior neighbours are solid (the
    interior problem) and rejected (-2) when one of them is fluid."""
    x = W.uniform_grid(12)
    Z, Y, X = W.mesh(x, x, x)
    ball = np.broadcast_to(0.3 - np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2), (12, 12, 12)).copy()
    one = np.ones_like(ball)
    P = oracle.Problem(x, x, x, ball, one, one)            # fluid inside the ball only
    assert P.info()["n_unknown"] > 0
    bad = ball.copy()
    bad[1:-1, 1, 1:-1] = 1.0                               # a fluid layer next to the y = 0 wall
    with pytest.raises(oracle.OracleError) as e:
        oracle.Problem(x, x, x, bad, one, one)
    assert e.value.code == -2
