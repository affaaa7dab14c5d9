"""Eigenvalue spectra of the discrete operators (Sec. 3.1): the compact operator B on the
unknowns, and B M with the preconditioner M (either inner solver of K).

The matrices are assembled column by column from the library's own operators (cps_apply,
cps_precond on unit vectors, FP64), so the spectra are those of what the GPU solves; the
eigenvalues are then computed densely on the host (numpy).  This is meant for small grids:
the paper's case is a uniform 21^3 grid, 6859 unknowns, with and without a sphere of radius
0.2 at the centre, eigenvalues scaled by dx^2.

Usage::

    python -m paper_1901_08269_amd.spectra --n 21 [--sphere 0.2] [--precond multigrid]
"""
import argparse
import json

import numpy as np

from . import Solver
from . import workloads as W


def unknown_nodes(solver):
    """Flat indices of the unknown (fluid interior) nodes."""
    _, t = solver.rhs_and_types()
    t = t.detach().cpu().numpy().ravel()
    return np.flatnonzero((t == 1) | (t == 2))


def assemble(solver, which="B"):
    """Dense matrix on the unknowns of B (which = "B") or of the preconditioner M ("M"),
    one operator application per column."""
    import torch
    nodes = unknown_nodes(solver)
    n = len(nodes)
    cols = np.empty((n, n))
    e = torch.zeros(solver.shape, dtype=torch.float64, device="cuda")
    flat = e.view(-1)
    idx = torch.as_tensor(nodes, device="cuda")
    for j, node in enumerate(nodes):
        flat[node] = 1.0
        y = solver.apply(e) if which == "B" else solver.precond(e)
        cols[:, j] = y.view(-1)[idx].cpu().numpy()
        flat[node] = 0.0
    return cols


def spectra(n=21, sphere=0.2, precond=None):
    """Eigenvalues of dx^2 B and of B M on a uniform n^3 grid (walls included), with a sphere
    of the given radius at the centre (None: no body)."""
    x = W.uniform_grid(n)
    bodies = [W.Sphere((0.5, 0.5, 0.5), sphere)] if sphere else []
    phi = W.union_level(bodies, x, x, x) if bodies else np.ones((n, n, n))
    one = np.ones((n, n, n))
    S = Solver(x, x, x, phi, one, one, precond=precond)
    B = assemble(S, "B")
    h2 = (x[1] - x[0]) ** 2
    lam = np.linalg.eigvals(B * h2)
    out = {"n": n, "sphere": sphere, "unknowns": int(B.shape[0]), "eig_B_dx2": lam}
    if precond is not None:
        M = assemble(S, "M")
        out["eig_BM"] = np.linalg.eigvals(B @ M)
    S.close()
    return out


def summary(lam):
    """Extent of a spectrum: real-part range, largest |imaginary part|, complex count."""
    return {"re_min": float(lam.real.min()), "re_max": float(lam.real.max()),
            "im_abs_max": float(np.abs(lam.imag).max()),
            "n_complex": int(np.sum(np.abs(lam.imag) > 1e-9 * np.abs(lam).max()))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=21)
    ap.add_argument("--sphere", type=float, default=0.2, help="sphere radius; 0: no body")
    ap.add_argument("--precond", choices=("chebyshev", "multigrid"), default=None)
    a = ap.parse_args(argv)
    r = spectra(a.n, a.sphere or None, a.precond)
    rep = {"n": r["n"], "sphere": r["sphere"], "unknowns": r["unknowns"], "B_dx2": summary(r["eig_B_dx2"])}
    if "eig_BM" in r:
        lam = r["eig_BM"]
        rep["BM"] = dict(summary(lam), abs_dev_from_1_max=float(np.abs(lam - 1).max()))
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
