"""Pins of the network oracle (oracle/net_oracle.c): the 3x3x3 convolution against torch's
CPU conv3d (an independent library routine), its backward against finite differences and
against torch autograd, the whole network's gradient against central differences, and the
BF16 rounding against the format's definition."""
import numpy as np
import pytest
import torch

from oracle import net


def test_conv3_matches_torch():
    rng = np.random.Generator(np.random.PCG64(0))
    x = rng.standard_normal((2, 5, 6, 6, 6))
    W = rng.standard_normal((7, 5, 3, 3, 3))
    b = rng.standard_normal(7)
    ref = torch.nn.functional.conv3d(torch.tensor(x), torch.tensor(W), torch.tensor(b), padding=1).numpy()
    np.testing.assert_allclose(net.conv3(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_conv3_backward_matches_autograd():
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.standard_normal((2, 4, 5, 5, 5))
    W = rng.standard_normal((3, 4, 3, 3, 3))
    g = rng.standard_normal((2, 3, 5, 5, 5))
    tx, tW, tb = (torch.tensor(v, requires_grad=True) for v in (x, W, np.zeros(3)))
    (torch.nn.functional.conv3d(tx, tW, tb, padding=1) * torch.tensor(g)).sum().backward()
    din, dW, db = net.conv3_bwd(x, W, g)
    np.testing.assert_allclose(din, tx.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, tW.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_network_gradient_finite_differences():
    ch = (4, 4, 8, 8)
    rng = np.random.Generator(np.random.PCG64(2))
    npar = net.param_count(ch, 3)
    params = rng.standard_normal(npar) * 0.3
    inp = rng.standard_normal((2, 3, 8, 8, 8))
    tgt = rng.standard_normal((2, 8, 8, 8))
    mask = (rng.random((2, 8, 8, 8)) > 0.2).astype(float)
    loss, _, g = net.run(params, inp, tgt, mask, ch=ch, bf16=False)
    idx = rng.choice(npar, 40, replace=False)
    for q in idx:
        h = 1e-6 * max(1.0, abs(params[q]))
        pp, pm = params.copy(), params.copy()
        pp[q] += h
        pm[q] -= h
        fd = (net.run(pp, inp, tgt, mask, ch=ch, bf16=False, grad=False)[0] -
              net.run(pm, inp, tgt, mask, ch=ch, bf16=False, grad=False)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-5 * max(1e-3, abs(fd)), (q, fd, g[q])


def test_network_matches_torch_composition():
    # the same architecture written with torch ops (CPU, float64) gives the same loss/grad
    ch = (4, 6, 8, 8)
    rng = np.random.Generator(np.random.PCG64(3))
    npar = net.param_count(ch, 3)
    params = rng.standard_normal(npar) * 0.2
    inp = rng.standard_normal((1, 3, 8, 8, 8))
    tgt = rng.standard_normal((1, 8, 8, 8))
    loss, pred, g = net.run(params, inp, tgt, None, ch=ch, bf16=False)
    P = torch.tensor(params, requires_grad=True)
    dims = [(3, ch[0]), (ch[0], ch[0]), (ch[0], ch[1]), (ch[1], ch[1]), (ch[1], ch[2]), (ch[2], ch[2]),
            (ch[2], ch[3]), (ch[3], ch[3]), (ch[3] + ch[2], ch[2]), (ch[2], ch[2]), (ch[2] + ch[1], ch[1]),
            (ch[1], ch[1]), (ch[1] + ch[0], ch[0]), (ch[0], ch[0])]
    o, layers = 0, []
    for ci, co in dims:
        Wl = P[o:o + co * ci * 27].reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        layers.append((Wl, P[o:o + co]))
        o += co
    hw, hb = P[o:o + ch[0]], P[o + ch[0]]
    F = torch.nn.functional

    def c(xx, L):
        return F.relu(F.conv3d(xx, layers[L][0], layers[L][1], padding=1))

    x = torch.tensor(inp)
    s0 = c(c(x, 0), 1)
    s1 = c(c(F.avg_pool3d(s0, 2), 2), 3)
    s2 = c(c(F.avg_pool3d(s1, 2), 4), 5)
    bt = c(c(F.avg_pool3d(s2, 2), 6), 7)
    up = lambda t: t.repeat_interleave(2, 2).repeat_interleave(2, 3).repeat_interleave(2, 4)
    d2 = c(c(torch.cat([up(bt), s2], 1), 8), 9)
    d1 = c(c(torch.cat([up(d2), s1], 1), 10), 11)
    d0 = c(c(torch.cat([up(d1), s0], 1), 12), 13)
    p = (d0 * hw.reshape(1, -1, 1, 1, 1)).sum(1) + hb
    L = ((p - torch.tensor(tgt)) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) <= 1e-12 * abs(loss)
    np.testing.assert_allclose(pred, p.detach().numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(g, P.grad.numpy(), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("v", [1.0, 1.00390625, 1.005859375, -3.14159, 1e-30, 65504.0, 0.0])
def test_bf16_rounding(v):
    # round to nearest even on the top 16 bits of the binary32 encoding
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).item()
    assert net.bf16(v) == ref
