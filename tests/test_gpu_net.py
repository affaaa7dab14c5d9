"""GPU tests of the learned warm start: the network's forward and backward kernels (BF16
MFMA) against the plain-loop oracle, training, save/load, the fine/coarse transfers, and
what the trained network gains over a zero initial guess."""
import os

import numpy as np
import pytest

import oracle.net as onet
import paper_1901_08269_amd as cps
from paper_1901_08269_amd import learned
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu

CH = (16, 32, 48, 64)


def _batch(nc, B, seed):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    inp = torch.tensor(rng.standard_normal((B, 3, nc, nc, nc)), dtype=torch.float32, device="cuda")
    tgt = torch.tensor(rng.standard_normal((B, nc, nc, nc)), dtype=torch.float32, device="cuda")
    msk = torch.tensor((rng.random((B, nc, nc, nc)) > 0.3).astype(np.float32), device="cuda")
    return inp, tgt, msk


# Bars for the BF16 network (both sides round weights, inputs, stored activations and the
# gradient entering each layer's backward pass to BF16 at the same places; they differ in
# FP32 vs FP64 accumulation and its order, which can move a stored BF16 value by one unit of
# its last place, 2^-8 relative): the prediction's and each parameter tensor's gradient's
# max-abs difference relative to that tensor's max.
PRED_BAR = 1e-2
GRAD_BAR = 2e-2


@pytest.mark.parametrize("nc,B", [(8, 2), (16, 1)])
def test_forward_backward_vs_oracle(nc, B):
    print(f"[case] net nc={nc} B={B}", flush=True)
    m = learned.Model(nc, batch=B, seed=7)
    inp, tgt, msk = _batch(nc, B, 11)
    loss = m.train_step(inp, tgt, msk, update=False)
    pred = m.forward(inp).cpu().numpy()
    w, g = m.params(grads=True)
    assert onet.param_count(CH, 3) == m.nparam
    loss_ref, pred_ref, g_ref = onet.run(w.astype(np.float64), inp.cpu().numpy().astype(np.float64),
                                         tgt.cpu().numpy().astype(np.float64), msk.cpu().numpy().astype(np.float64),
                                         ch=CH, bf16=True)
    rel_pred = np.max(np.abs(pred - pred_ref)) / np.max(np.abs(pred_ref))
    print(f"loss {loss:.6e} / {loss_ref:.6e}; prediction max rel {rel_pred:.2e}")
    assert abs(loss - loss_ref) <= 2e-3 * abs(loss_ref)
    assert rel_pred <= PRED_BAR
    # every parameter tensor's gradient on its own scale
    worst = 0.0
    for name, sl in onet.layer_slices(CH, 3):
        ref = g_ref[sl]
        err = float(np.max(np.abs(g[sl] - ref)) / np.max(np.abs(ref)))
        print(f"  {name:7s} {sl.stop - sl.start:7d} params  grad max rel {err:.2e}")
        assert np.max(np.abs(ref)) > 0.0, name
        worst = max(worst, err)
        assert err <= GRAD_BAR, name
    print(f"worst tensor {worst:.2e}")


def test_adam_steps_vs_oracle():
    """Two training steps with the Adam update: the parameters after each step against the
    oracle's Adam (Kingma & Ba, Algorithm 1) applied to the same starting parameters and the
    gradients the library reports for each step."""
    import oracle.warmstart as ows
    print("[case] adam two steps nc=8", flush=True)
    m = learned.Model(8, batch=2, seed=5)
    inp, tgt, msk = _batch(8, 2, 13)
    w0 = m.params().astype(np.float64)
    lr = 1e-3
    ws, gs = [], []
    for _ in range(2):
        m.train_step(inp, tgt, msk, lr=lr, update=True)
        w, g = m.params(grads=True)
        ws.append(w.astype(np.float64))
        gs.append(g.astype(np.float64))
    refs = ows.adam(w0, gs, lr=lr)
    for q, (w, ref) in enumerate(zip(ws, refs)):
        err = np.abs(w - ref)
        bar = 2e-7 * np.abs(ref) + 1e-4 * lr
        print(f"step {q + 1}: max |w - w_ref| {err.max():.2e}, max moved {np.max(np.abs(ref - w0)):.2e}")
        assert np.all(err <= bar)
    # the first step moves every parameter with a clear gradient by lr (m^ = g, v^ = g^2)
    live = np.abs(gs[0]) > 1e-5
    assert live.sum() > 1000
    np.testing.assert_allclose(np.abs(ws[0] - w0)[live], lr, rtol=1e-2)


def test_training_reduces_loss_and_save_load(tmp_path):
    m = learned.Model(16, batch=4, seed=2)
    inp, tgt, _ = _batch(16, 4, 3)
    tgt = inp[:, 0] * 0.5 + 0.2 * inp[:, 2]      # a learnable linear map of the inputs
    l0 = m.train_step(inp, tgt, update=False)
    for _ in range(60):
        m.train_step(inp, tgt, lr=3e-3)
    l1 = m.train_step(inp, tgt, update=False)
    assert l1 < 0.5 * l0, (l0, l1)
    path = str(tmp_path / "w.bin")
    m.save(path)
    m2 = learned.Model(16, batch=4, seed=99)
    m2.load(path)
    p1, p2 = m.forward(inp), m2.forward(inp)
    assert float((p1 - p2).abs().max()) == 0.0


def test_checkpoint_resumes_training_exactly(tmp_path):
    """A checkpoint carries Adam's step count and moments: training resumed from it takes the
    same steps as uninterrupted training, bit for bit (the kernels reduce in a fixed order).
    A weights-only file restarts Adam, which then takes a different step."""
    inp, tgt, msk = _batch(8, 2, 11)
    m = learned.Model(8, batch=2, seed=5)
    for _ in range(3):
        m.train_step(inp, tgt, msk, lr=2e-3)
    ck = str(tmp_path / "ck.bin")
    wo = str(tmp_path / "w.bin")
    m.save_checkpoint(ck)
    m.save(wo)
    assert os.path.getsize(ck) > 2.9 * os.path.getsize(wo)
    for _ in range(2):
        m.train_step(inp, tgt, msk, lr=2e-3)
    ref = m.params()
    r = learned.Model(8, batch=2, seed=77)
    r.load(ck)
    for _ in range(2):
        r.train_step(inp, tgt, msk, lr=2e-3)
    got = r.params()
    print(f"resumed vs uninterrupted: max |dw| {np.abs(got - ref).max():.3e}")
    assert np.array_equal(got, ref)
    f = learned.Model(8, batch=2, seed=77)
    f.load(wo)
    for _ in range(2):
        f.train_step(inp, tgt, msk, lr=2e-3)
    assert not np.array_equal(f.params(), ref)
    bad = str(tmp_path / "bad.bin")
    with open(bad, "wb") as fh:
        fh.write(b"CPSNET03" + bytes(64))
    with pytest.raises(cps.CpsError):
        r.load(bad)


def test_restrict_all_channels_vs_oracle():
    """The network input of a problem (cell means of f, phi, g with the sigma scaling, and the
    target's cell means of u) against the oracle's restriction, every channel."""
    import torch
    import oracle.warmstart as ows
    N = 32
    print(f"[case] restrict N={N}", flush=True)
    w = W.sphere_sin(N, beta=1.2, r=0.2)
    S = cps.Solver.from_workload(w)
    m = learned.Model(N // 4, batch=1)
    u = torch.tensor(w.u_exact, device="cuda")
    inp, tgt, sigma = m.restrict(S, u)
    ref, sig = ows.restrict_inputs(w.f, w.phi, w.g, N // 4)
    assert abs(sigma - sig) <= 1e-13 * sig
    got = inp[0].cpu().numpy().astype(np.float64)
    for c in range(3):
        err = np.max(np.abs(got[c] - ref[c])) / np.max(np.abs(ref[c]))
        print(f"channel {c}: max rel {err:.2e}")
        assert err <= 2e-7          # an FP32 rounding of an FP64 mean
    assert np.max(np.abs(ref[1])) < 1.0 and np.min(ref[1]) < 0.0 < np.max(ref[1])   # phi unclamped, both signs
    tref = ows.restrict_target(w.u_exact, w.phi, w.g, sig, N // 4)
    assert np.any(w.phi[1:-1, 1:-1, 1:-1] <= 0.0)    # the body's nodes take g
    assert np.max(np.abs(tgt[0].cpu().numpy() - tref)) <= 2e-7 * np.max(np.abs(tref))


def test_prolong_vs_oracle():
    """cps_model_predict = sigma x trilinear (index-space) prolongation of the network's
    prediction: the library's u0 against the oracle's prolongation of the prediction the
    library's forward pass gives for the same input (the kernels are deterministic)."""
    import oracle.warmstart as ows
    N = 32
    print(f"[case] prolong N={N}", flush=True)
    w = W.sphere_sin(N, beta=1.2, r=0.2)
    S = cps.Solver.from_workload(w)
    m = learned.Model(N // 4, batch=1, seed=4)
    inp, _, sigma = m.restrict(S)
    pred = m.forward(inp)[0].cpu().numpy().astype(np.float64)
    u0 = m.predict(S).cpu().numpy()
    ref = ows.prolong(pred, sigma, u0.shape)
    err = np.max(np.abs(u0 - ref)) / np.max(np.abs(ref))
    print(f"prolongation max rel {err:.2e}")
    assert err <= 1e-12


def test_predict_fields_matches_predict():
    """cps_model_predict_fields (the fields themselves, queued on a stream of the caller's, no
    solver) gives cps_model_predict's u0 bit for bit, on a side stream and on the current one;
    a grid that is not 4 nc points a side is refused."""
    import torch
    N = 32
    print(f"[case] predict_fields N={N}", flush=True)
    w = W.sphere_sin(N, beta=1.2, r=0.2)
    S = cps.Solver.from_workload(w)
    m = learned.Model(N // 4, batch=1, seed=5)
    ref = m.predict(S).cpu().numpy()
    fields = [torch.as_tensor(getattr(w, k), dtype=torch.float64).cuda().contiguous() for k in ("phi", "g", "f")]
    side = torch.cuda.Stream()
    u_side = m.predict_fields(*fields, side)
    side.synchronize()
    u_cur = m.predict_fields(*fields, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(u_side.cpu().numpy(), ref)
    assert np.array_equal(u_cur.cpu().numpy(), ref)
    small = [t[:-4, :-4, :-4].contiguous() for t in fields]
    with pytest.raises(Exception):
        m.predict_fields(*small, side)
    side.synchronize()
    S.close()


def test_headline_mixed_learned_vs_oracle_samples():
    """The benchmark path: 256^3, 8 spheres, mixed precision from the shipped network's warm
    start.  At tol 1e-10 both residual norms meet the bound; at tol 1e-13 the solution matches
    the FP64 oracle (solved to 1e-13) to <= 1e-9 relative max-norm on the stored samples.
    (At 1e-10 the iteration error of this system, condition ~1e7, is ~1e-8 relative.)"""
    from gold import samples
    nodes, vals, umax = samples("oracle_spheres8_256.txt")
    w = W.spheres8(256)
    print("[case] spheres8 256 mixed + learned warm start", flush=True)
    S = cps.Solver.from_workload(w, precision="mixed")
    ws_ = learned.load_default(256)
    u0 = ws_.predict(S)
    u, st = S.solve(1e-10, u0=u0)
    print(f"tol 1e-10: {st['iters']} iterations, alpha {st['warm_alpha']:.3f}, rel res {st['rel_residual']:.2e}")
    assert st["rel_residual"] <= 1e-10 and st["rel_residual_jacobi"] <= 1e-10
    assert st["warm_alpha"] > 0.0
    rel10 = np.max(np.abs(u.reshape(-1).cpu().numpy()[nodes] - vals)) / umax
    u, st = S.solve(1e-13, u0=u0)
    assert st["rel_residual"] <= 1e-13 and st["rel_residual_jacobi"] <= 1e-13
    rel = np.max(np.abs(u.reshape(-1).cpu().numpy()[nodes] - vals)) / umax
    print(f"vs oracle samples: tol 1e-10 {rel10:.2e}, tol 1e-13 {rel:.2e} ({st['iters']} iterations)")
    assert rel <= 1e-9
    S.close()


@pytest.mark.slow
def test_warm_start_saves_iterations():
    """Train on 48 solver-generated instances of the eight-sphere family at 64^3 (a new body
    configuration and smooth solution per seed) and check the warm start on 4 unseen seeds:
    fewer iterations on average, the same solution to the solver's tolerance."""
    N = 64
    X, Y = learned.generate("spheres8", N, list(range(1000, 1048)))
    m = learned.Model(N // 4, batch=8, seed=1)
    hist, steps, secs = learned.train(m, X, Y, epochs=25, lr=3e-3)
    assert hist[-1] < 0.2 * hist[0]
    ev = learned.Model(N // 4, batch=1)
    ev.set_params(m.params())
    rows = learned.warm_start_gain(ev, "spheres8", N, [100000, 100001, 100002, 100003])
    saved = np.array([r["iters_zero"] - r["iters_warm"] for r in rows])
    print("iterations saved per test instance:", saved.tolist())
    assert saved.mean() > 0
    assert max(r["diff"] for r in rows) <= 1e-8


@pytest.mark.slow
def test_warm_start_star_family_not_worse():
    """The star-body family (random Fourier f, g = 0): a 4x-coarse representation cannot carry
    the fine-scale part of its solution, so the learned start saves little or nothing there
    (even the restriction of the exact solution does not).  The residual-based scaling in
    cps_solve keeps its start no worse than zero in the residual norm, so on average it costs
    at most an iteration (single seeds move by one or two either way: BiCGSTAB's iteration
    count is that sensitive to the start), and the solution is the same."""
    N = 64
    X, Y = learned.generate("star", N, list(range(48)))
    m = learned.Model(N // 4, batch=8, seed=1)
    hist, steps, secs = learned.train(m, X, Y, epochs=25, lr=3e-3)
    assert hist[-1] < 0.2 * hist[0]
    ev = learned.Model(N // 4, batch=1)
    ev.set_params(m.params())
    rows = learned.warm_start_gain(ev, "star", N, [100000, 100001, 100002, 100003])
    saved = np.array([r["iters_zero"] - r["iters_warm"] for r in rows])
    print("iterations saved per test instance:", saved.tolist())
    assert saved.mean() >= -1.0
    assert max(r["diff"] for r in rows) <= 1e-8
