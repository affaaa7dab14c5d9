"""Oracle of the multigrid preconditioner for K (test infrastructure: only tests, smoke
checks and the benchmark's CPU baseline use it).

The paper preconditions BiCGSTAB with the second-order operator K (Sec. 3.3), applied
approximately by an inner iterative solver, and says another inner solver may be used.
This is a geometric multigrid V-cycle for K.  It is written out plainly: every operation is
a loop-free numpy expression or a call of the C oracle (K rows, the Chebyshev-Jacobi
smoother), so that it can be checked by eye against this definition:

* Levels.  Level 0 is the problem's grid.  A coarser level keeps, along every axis, the
  even-indexed points and the last point (a wall); its level set is the finer level set at
  those nodes, and its K (Eqs. 2ndorder_coef, A7, with Shortley-Weller rows at nodes next
  to the body, Eqs. 2ndorder_coef_mod, A7_mod) is built on its own coordinates.  Coarsening
  stops after `levels` levels, when an axis would have fewer than `min_points` points, or
  once a level has at most `coarse_interior` interior points.
* Transfer.  Prolongation P is the tensor product of 1D linear interpolation in the
  physical coordinate: a fine node that is a coarse node takes its value, a fine node
  between coarse nodes a and b takes (1 - w) e_a + w e_b with w = (x - x_a) / (x_b - x_a).
  Restriction is P^T with each coarse row divided by its sum (constants are kept).  Only
  unknown (fluid interior) nodes carry values; others are 0 on every level.
* V-cycle on level l for K_l x = rho: `nu` Chebyshev-Jacobi steps from x = 0 on the
  spectrum interval [smooth_lo, 2] of diag(K)^-1 K; residual r = rho - K_l x; x += P (V-cycle
  on level l + 1 of R r) at the regular unknown nodes (an irregular node, next to the body,
  gets no coarse correction: the coarse grid sees the interface elsewhere, and its
  interpolated correction there is what the post-smoothing must undo); `nu` more steps from x.  On the coarsest level: `coarse_steps`
  steps from 0 on [lambda_1, 2], lambda_1 = (1/3) sum_d (1 - cos(pi / (n_d - 1))).

The cycle is a fixed linear map of rho, as right-preconditioned BiCGSTAB requires.
"""
import numpy as np

import oracle

HI = 2.0


def coarse_indices(n):
    """Indices of a fine axis of n points kept on the next coarser level."""
    idx = list(range(0, n - 1, 2))
    if idx[-1] != n - 1:
        idx.append(n - 1)
    return np.array(idx)


def interp_1d(xf, xc, idx):
    """(left coarse index, weight of the right coarse node) for every fine point."""
    a = np.searchsorted(idx, np.arange(len(xf)), side="right") - 1
    a = np.minimum(a, len(xc) - 2)
    w = (xf - xc[a]) / (xc[a + 1] - xc[a])
    return a, w


def prolong(ec, ax):
    """Tensor-product linear interpolation of a coarse field (nz, ny, nx) to the fine grid."""
    out = ec
    for axis, (a, w) in zip((2, 1, 0), ax):       # x, y, z
        lo = np.take(out, a, axis=axis)
        hi = np.take(out, a + 1, axis=axis)
        sh = [1, 1, 1]
        sh[axis] = len(w)
        wv = w.reshape(sh)
        out = (1.0 - wv) * lo + wv * hi
    return out


def restrict(rf, ax, shape_c):
    """P^T rf with each coarse row divided by its row sum."""
    out = rf
    for axis, (a, w), nc in zip((2, 1, 0), ax, (shape_c[2], shape_c[1], shape_c[0])):
        moved = np.moveaxis(out, axis, 0)
        acc = np.zeros((nc,) + moved.shape[1:])
        np.add.at(acc, a, (1.0 - w)[(slice(None),) + (None,) * (moved.ndim - 1)] * moved)
        np.add.at(acc, a + 1, w[(slice(None),) + (None,) * (moved.ndim - 1)] * moved)
        wsum = np.zeros(nc)
        np.add.at(wsum, a, 1.0 - w)
        np.add.at(wsum, a + 1, w)
        acc /= wsum[(slice(None),) + (None,) * (moved.ndim - 1)]
        out = np.moveaxis(acc, 0, axis)
    return out


def lambda_1(shape):
    return sum(1.0 - np.cos(np.pi / (n - 1)) for n in shape) / 3.0


class Multigrid:
    def __init__(self, x, y, z, phi, levels=16, nu=2, smooth_lo=0.2, coarse_steps=8, min_points=9,
                 coarse_interior=4096):
        self.nu, self.smooth_lo, self.coarse_steps = nu, smooth_lo, coarse_steps
        self.lv = []
        xs, phis = (np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)), np.asarray(phi, float)
        for l in range(levels):
            P = oracle.Problem.k_only(xs[0], xs[1], xs[2], phis)
            t = P.types()
            self.lv.append({"P": P, "x": xs, "unk": ((t == 1) | (t == 2)).astype(float), "reg": (t == 1).astype(float),
                            "shape": phis.shape})
            interior = np.prod([len(c) - 2 for c in xs])
            if l + 1 == levels or min(len(c) for c in xs) < 2 * min_points - 1 or interior <= coarse_interior:
                break
            idx = [coarse_indices(len(c)) for c in xs]
            xc = tuple(c[i] for c, i in zip(xs, idx))
            self.lv[-1]["ax"] = [interp_1d(xf, xcc, i) for xf, xcc, i in zip(xs, xc, idx)]
            phis = np.ascontiguousarray(phis[np.ix_(idx[2], idx[1], idx[0])])
            xs = xc

    def vcycle(self, l, rho):
        L = self.lv[l]
        rho = rho * L["unk"]
        if l + 1 == len(self.lv):
            lo = lambda_1(L["shape"])
            return L["P"].smooth(rho, np.zeros_like(rho), self.coarse_steps, lo, HI) * L["unk"]
        x = L["P"].smooth(rho, np.zeros_like(rho), self.nu, self.smooth_lo, HI)
        r = (rho - L["P"].apply_K(x)) * L["unk"]
        rc = restrict(r, L["ax"], self.lv[l + 1]["shape"])
        ec = self.vcycle(l + 1, rc)
        x = x + prolong(ec, L["ax"]) * L["reg"]
        x = L["P"].smooth(rho, x, self.nu, self.smooth_lo, HI)
        return x * L["unk"]

    def apply(self, rho):
        return self.vcycle(0, np.asarray(rho, float))
