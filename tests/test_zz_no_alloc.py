"""cps_model_restrict_noalloc (the restriction for callers that cannot allocate) against
cps_model_restrict on the same problems: two calls in a row, the second on a smaller grid,
each output bit for bit (both run the same kernels in the same order)."""
import numpy as np
import pytest

import paper_1901_08269_amd as cps
from paper_1901_08269_amd import learned
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_restrict_noalloc_matches_restrict():
    import torch
    for N in (64, 32):
        print(f"[case] restrict_noalloc N={N}", flush=True)
        w = W.sphere_sin(N, beta=1.2, r=0.2)
        S = cps.Solver.from_workload(w)
        m = learned.Model(N // 4, batch=1)
        u = torch.tensor(w.u_exact, device="cuda")
        a_inp, a_tgt, a_sig = m.restrict(S, u)
        # outputs prefilled with NaN: every element must be written
        out = (torch.full_like(a_inp, float("nan")), torch.full_like(a_tgt, float("nan")))
        b_inp, b_tgt, b_sig = m.restrict(S, u, out=out, noalloc=True)
        assert b_sig == a_sig
        assert torch.equal(a_inp, b_inp) and torch.equal(a_tgt, b_tgt)
        assert np.isfinite(b_inp.cpu().numpy()).all()
        # without a target, as cps_model_predict calls it
        c_inp, _, c_sig = m.restrict(S, noalloc=True)
        assert c_sig == a_sig and torch.equal(c_inp, a_inp)
        m.close()
        S.close()
