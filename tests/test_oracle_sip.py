"""Pins of the oracle's strongly implicit procedure for K (oracle/cps_oracle.c,
orc_sip_factor / orc_sip_precond): with no partial cancellation (alpha = 0) L U is the
incomplete factorisation without fill, equal to K on K's pattern; with full cancellation
(alpha = 1) L U reproduces K on fields linear in the node index away from walls and
bodies, and with alpha = 0.5 it does not; the iteration is a fixed linear map that converges
to a dense direct solve of K."""
import numpy as np
import pytest

import oracle
from paper_1901_08269_amd import workloads as W


def _sphere_problem(n=14, r=0.23):
    w = W.sphere_sin(n - 2, beta=0.0, r=r)
    return oracle.Problem.from_workload(w)


def _dense(P, F):
    """Dense K, L (b, c, d and e on the diagonal) and U (unit diagonal, f, g, h) over the
    unknowns, and the unknown node list."""
    t = P.types().ravel()
    unk = np.nonzero((t == 1) | (t == 2))[0]
    pos = -np.ones(P.nn, np.int64)
    pos[unk] = np.arange(len(unk))
    nz, ny, nx = P.shape
    n = len(unk)
    K = np.zeros((n, n))
    L = np.zeros((n, n))
    U = np.eye(n)
    Fr = F.reshape(7, -1)
    offs = [0, -1, 1, -nx, nx, -nx * ny, nx * ny]
    for r, e in enumerate(unk):
        co = P.krow(e)
        for o, v in zip(offs, co):
            if pos[e + o] >= 0:
                K[r, pos[e + o]] += v
        b, c, d, ee, f, g, h = Fr[:, e]
        L[r, r] = ee
        for o, v in ((-nx * ny, b), (-nx, c), (-1, d)):
            if pos[e + o] >= 0:
                L[r, pos[e + o]] = v
            else:
                assert v == 0.0
        for o, v in ((1, f), (nx, g), (nx * ny, h)):
            if pos[e + o] >= 0:
                U[r, pos[e + o]] = v
            else:
                assert v == 0.0
    return K, L, U, unk, pos


def test_alpha0_is_ilu0():
    P = _sphere_problem()
    K, L, U, unk, pos = _dense(P, P.sip_factors(0.0))
    LU = L @ U
    pattern = K != 0.0
    np.testing.assert_allclose(LU[pattern], K[pattern], rtol=1e-13, atol=1e-13 * np.max(np.abs(K)))
    # the fill lies at the six positions B+E, B+N, S+E, S+T, W+N, W+T only
    nz, ny, nx = P.shape
    fill_offs = {-nx * ny + 1, -nx * ny + nx, -nx + 1, -nx + nx * ny, -1 + nx, -1 + nx * ny}
    rows, cols = np.nonzero(np.abs(LU - K) > 1e-12 * np.max(np.abs(K)))
    assert len(rows) > 0
    assert set((unk[cols] - unk[rows]).tolist()) <= fill_offs


def test_full_cancellation_exact_on_linear_fields():
    n = 12
    x = W.uniform_grid(n)
    w = W.polynomial_case(0, [], rng_seed=1, grids=(x, x, x))
    P = oracle.Problem.from_workload(w)
    nz, ny, nx = P.shape
    Kz, Jz, Iz = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = (0.3 + 1.7 * Iz - 0.6 * Jz + 2.2 * Kz).astype(float)
    inner = (Iz >= 2) & (Iz <= nx - 3) & (Jz >= 2) & (Jz <= ny - 3) & (Kz >= 2) & (Kz <= nz - 3)
    for alpha, exact in ((1.0, True), (0.5, False)):
        K, L, U, unk, pos = _dense(P, P.sip_factors(alpha))
        v = phi.ravel()[unk]
        d = (L @ (U @ v)) - K @ v
        rows = inner.ravel()[unk]
        err = np.max(np.abs(d[rows])) / np.max(np.abs(K @ v))
        if exact:
            assert err <= 1e-12, err
        else:
            assert err > 1e-3, err


def test_iteration_is_linear_and_converges_to_the_direct_solve():
    P = _sphere_problem(15, 0.25)
    rng = np.random.Generator(np.random.PCG64(4))
    t = P.types()
    unk = (t == 1) | (t == 2)
    a, b = rng.standard_normal(P.shape) * unk, rng.standard_normal(P.shape) * unk
    F = P.sip_factors(0.5)
    pa, pb = P.precond_sip(a, 8, factors=F), P.precond_sip(b, 8, factors=F)
    pab = P.precond_sip(2.0 * a - 3.0 * b, 8, factors=F)
    np.testing.assert_allclose(pab, 2.0 * pa - 3.0 * pb, rtol=0, atol=1e-12 * np.max(np.abs(pab)))
    assert np.all(pa[~unk] == 0.0)
    K, L, U, idx, pos = _dense(P, F)
    exact = np.linalg.solve(K, a.ravel()[idx])
    errs = [np.max(np.abs(P.precond_sip(a, m, factors=F).ravel()[idx] - exact)) / np.max(np.abs(exact))
            for m in (2, 8, 64)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 0.1 and errs[2] < 1e-9, errs
