"""The spectral tool (Sec. 3.1) on the GPU library's operators: the assembled B equals the
oracle's; on a uniform grid its spectrum is real and negative without a body and has
negative real parts with a sphere of radius 0.2 (the paper's 21^3 case runs from the
command line; the tests use 15^3 to keep the dense eigensolves short), and B M has positive
real parts with either inner solver of the preconditioner."""
import numpy as np
import pytest

import oracle
import paper_1901_08269_amd as cps
from paper_1901_08269_amd import spectra
from paper_1901_08269_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_assembled_B_matches_the_oracle():
    n = 13
    x = W.uniform_grid(n)
    phi = W.union_level([W.Sphere((0.5, 0.48, 0.52), 0.25)], x, x, x)
    one = np.ones((n, n, n))
    S = cps.Solver(x, x, x, phi, one, one)
    B = spectra.assemble(S, "B")
    ref, unk = oracle.Problem(x, x, x, phi, one, one).csr()
    assert np.array_equal(spectra.unknown_nodes(S), unk)
    ref = ref.toarray()
    assert np.max(np.abs(B - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("precond", ["chebyshev", "multigrid"])
@pytest.mark.parametrize("sphere", [None, 0.2])
def test_spectrum_of_B_and_BM(sphere, precond):
    print(f"[case] spectrum 15^3 sphere {sphere} {precond}", flush=True)
    r = spectra.spectra(15, sphere, precond=precond)
    lam = r["eig_B_dx2"]
    s = spectra.summary(lam)
    print(s, spectra.summary(r["eig_BM"]))
    assert s["re_max"] < 0.0
    if sphere is None:
        assert r["unknowns"] == 13 ** 3
        assert s["im_abs_max"] <= 1e-10 * np.abs(lam).max()     # symmetric: a real spectrum
    else:
        assert s["n_complex"] > 0                                 # the interface makes B non-normal
    assert np.all(r["eig_BM"].real > 0.0)
