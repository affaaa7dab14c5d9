"""Pins of the warm start's transfer and optimiser oracle (oracle/warmstart.py) against
what the mathematics fixes: block means of fields whose means have closed forms, a single
nonzero node, exactness of the index-space prolongation on trilinear fields with different
coefficients per axis, its constant extension beyond the outer cell centres, and Adam steps
computed by hand from Kingma & Ba's Algorithm 1."""
import numpy as np
import pytest

from oracle import warmstart as ws


def _idx(nc):
    n = 4 * nc + 2
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return k.astype(float), j.astype(float), i.astype(float)


def test_block_means_of_a_linear_field():
    # the mean of an arithmetic sequence is its middle value: nodes 1+4c .. 4+4c average to
    # 2.5 + 4c, so a + b i + c j + d k has cell means a + b (2.5 + 4cx) + c (2.5 + 4cy) + d (2.5 + 4cz)
    nc = 3
    K, J, I = _idx(nc)
    a = 0.7 + 2.0 * I - 0.3 * J + 5.0 * K
    cz, cy, cx = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    want = 0.7 + 2.0 * (2.5 + 4 * cx) - 0.3 * (2.5 + 4 * cy) + 5.0 * (2.5 + 4 * cz)
    np.testing.assert_allclose(ws.block_means(a, nc), want, rtol=0, atol=1e-12)


def test_block_means_single_node():
    # one node at (i, j, k) = (6, 1, 12) lies in cell (cx, cy, cz) = (1, 0, 2) and counts 1/64 there
    nc = 4
    a = np.zeros((4 * nc + 2,) * 3)
    a[12, 1, 6] = 64.0
    m = ws.block_means(a, nc)
    assert m[2, 0, 1] == 1.0
    assert np.count_nonzero(m) == 1
    # wall nodes never enter
    a[:] = 0.0
    a[0, :, :] = a[-1, :, :] = a[:, 0, :] = a[:, -1, :] = a[:, :, 0] = a[:, :, -1] = 1.0
    assert np.all(ws.block_means(a, nc) == 0.0)


def test_restrict_inputs_channels_and_sigma():
    nc = 2
    n = 4 * nc + 2
    f = np.full((n, n, n), 3.0 * np.pi ** 2 * 2.0)   # f / 3 pi^2 = 2
    g = np.full((n, n, n), 1.5)
    # sigma = sqrt(1.5^2 + 2^2) = 2.5
    phi = np.full((n, n, n), -1.0)
    phi[..., 5:] = 40.0                               # cells with cx = 1 hold phi = 40
    inp, sigma = ws.restrict_inputs(f, phi, g, nc)
    assert sigma == pytest.approx(2.5, rel=1e-15)
    np.testing.assert_allclose(inp[0], 2.0 / 2.5, rtol=1e-15)
    np.testing.assert_allclose(inp[2], 1.5 / 2.5, rtol=1e-15)
    # phi channel: clamp(mean * nc / 8): -1 * 2 / 8 = -0.25 in cx = 0; 40 * 2 / 8 = 10 -> 1 in cx = 1
    np.testing.assert_allclose(inp[1][..., 0], -0.25, rtol=1e-15)
    np.testing.assert_allclose(inp[1][..., 1], 1.0, rtol=0)
    # the solution is linear in (f, g): scaling both leaves the input unchanged and scales sigma
    inp2, sigma2 = ws.restrict_inputs(4.0 * f, phi, 4.0 * g, nc)
    assert sigma2 == pytest.approx(4.0 * sigma, rel=1e-15)
    np.testing.assert_allclose(inp2, inp, rtol=1e-15)
    # a zero problem keeps sigma = 1
    assert ws.scale_sigma(np.zeros(8), np.zeros(8)) == 1.0
    # the target is the cell mean of u / sigma, with g in place of u where phi <= 0
    u = 2.0 * f / (3.0 * np.pi ** 2)                  # 4 everywhere
    np.testing.assert_allclose(ws.restrict_target(u, np.ones_like(phi), g, 2.5, nc), 4.0 / 2.5, rtol=1e-15)
    # cells with cx = 0 lie in phi = -1: their target is g = 1.5 (not u = 4, not 0)
    t = ws.restrict_target(u, phi, g, 2.5, nc)
    np.testing.assert_allclose(t[..., 0], 1.5 / 2.5, rtol=1e-15)
    np.testing.assert_allclose(t[..., 1], 4.0 / 2.5, rtol=1e-15)
    # a block with one node inside the body: (63 u + g) / 64
    phi2 = np.ones_like(phi)
    phi2[1, 1, 1] = -0.5
    t2 = ws.restrict_target(u, phi2, g, 1.0, nc)
    assert t2[0, 0, 0] == pytest.approx((63 * 4.0 + 1.5) / 64, rel=1e-15)
    assert t2[1, 1, 1] == pytest.approx(4.0, rel=1e-15)


def test_prolong_exact_on_trilinear_fields():
    # a coarse field trilinear in the cell index with a different coefficient per axis is
    # reproduced exactly at every fine node between the outer cell centres, at coarse
    # coordinate s = (i - 2.5) / 4 per axis; outside them the value is that at the clamped s
    nc = 5
    cz, cy, cx = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")

    def F(sx, sy, sz):
        return 1.0 + 0.5 * sx - 2.0 * sy + 3.0 * sz + 0.25 * sx * sy - 0.75 * sy * sz + 0.1 * sx * sy * sz

    p = F(cx, cy, cz)
    shape = (4 * nc + 2, 4 * nc + 1, 4 * nc + 2)        # the y axis one node short: a ragged shape
    u = ws.prolong(p, 2.0, shape)
    K, J, I = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    s = [np.clip((A - 2.5) / 4.0, 0.0, nc - 1.0) for A in (I, J, K)]
    np.testing.assert_allclose(u, 2.0 * F(*s), rtol=0, atol=1e-12)


def test_prolong_constant_and_extension():
    nc = 3
    u = ws.prolong(np.full((nc, nc, nc), -1.25), 1.0, (14, 14, 14))
    np.testing.assert_allclose(u, -1.25, rtol=0, atol=1e-15)
    # one nonzero cell: its value reaches fine nodes within one cell spacing (4 fine nodes) of its centre,
    # and nodes 0, 1, 2 (before cell 0's centre at 2.5) carry cell 0's value unchanged
    p = np.zeros((nc, nc, nc))
    p[0, 0, 0] = 1.0
    u = ws.prolong(p, 1.0, (14, 14, 14))
    assert u[0, 0, 0] == 1.0 and u[2, 2, 2] == 1.0
    assert u[3, 2, 2] == pytest.approx(1.0 - 0.125)            # s = 0.125 in z
    assert np.all(u[7:, :, :] == 0.0) and np.all(u[:, :, 7:] == 0.0)


def test_adam_hand_computed():
    # step 1 from zero moments: m^ = g, v^ = g^2, so the step is lr g / (|g| + eps)
    w1, w2 = ws.adam([1.0, -2.0, 0.5], [[1.0, 1.0, -4.0], [1.0, -1.0, -4.0]], lr=0.01, eps=0.0)
    np.testing.assert_allclose(w1, [1.0 - 0.01, -2.0 - 0.01, 0.5 + 0.01], rtol=1e-15)
    # step 2, constant gradient: m_2 = 0.19 g, m^ = g; v_2 = 0.001999 g^2, v^ = g^2: another lr step
    assert w2[0] == pytest.approx(0.99 - 0.01, rel=1e-14)
    assert w2[2] == pytest.approx(0.51 + 0.01, rel=1e-14)
    # step 2 with a sign flip: m_2 = 0.9 * 0.1 - 0.1 = -0.01, m^ = -0.01 / 0.19; v^ = 1
    assert w2[1] == pytest.approx(-2.01 + 0.01 * (0.01 / 0.19), rel=1e-14)


def test_adam_invariances():
    rng = np.random.Generator(np.random.PCG64(0))
    g = [rng.standard_normal(6) for _ in range(4)]
    base = ws.adam(np.zeros(6), g, lr=1e-3, eps=0.0)
    # invariant to a positive rescaling of every gradient (eps = 0)
    scaled = ws.adam(np.zeros(6), [7.5 * x for x in g], lr=1e-3, eps=0.0)
    np.testing.assert_allclose(scaled[-1], base[-1], rtol=1e-12, atol=1e-18)
    # the step bound of Kingma & Ba (Sec. 2.1): |step| <= lr (1 - b1) / sqrt(1 - b2) when 1 - b1 > sqrt(1 - b2)
    prev = np.zeros(6)
    for w in base:
        assert np.max(np.abs(w - prev)) <= 1e-3 * 0.1 / np.sqrt(0.001) * (1 + 1e-12)
        prev = w
    # eps bounds the step of a vanishing gradient: zero gradient -> no move
    z = ws.adam(np.ones(3), [np.zeros(3)], lr=0.1)
    np.testing.assert_array_equal(z[0], np.ones(3))
