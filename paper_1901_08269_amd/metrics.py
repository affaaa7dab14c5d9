"""Measurement helpers: the paper's FLOP model and order estimator, and the byte model of
the GPU sweeps used for the roofline figures.

These hold no solver arithmetic; they turn counts and timings into reported numbers.
"""
from __future__ import annotations

import math


def flops_per_iteration(n_points: int, n_irr: int, iter_prec: int = 8) -> float:
    """FLOPs of one preconditioned BiCGSTAB outer iteration, Table flop (Sec. 3.4):
    (126 + 80 iter_prec) N + 432 N_irr."""
    return (126.0 + 80.0 * iter_prec) * n_points + 432.0 * n_irr


def flop_extra_percent(n_points: int, n_irr: int, iter_prec: int = 8) -> float:
    """Eq. (flop): FLOP_extra(%) = N_irr / N * 432 / (126 + 80 iter_prec) * 100.

    The paper's tables are reproduced with N = n^3, the total number of grid points."""
    return n_irr / n_points * 432.0 / (126.0 + 80.0 * iter_prec) * 100.0


def order_estimate(e1: float, e2: float, n1: int, n2: int) -> float:
    """Eq. (order): p = log(E_n1 / E_n2) / log((n2 - 1) / (n1 - 1)), n = points per direction."""
    return math.log(e1 / e2) / math.log((n2 - 1) / (n1 - 1))


# Algorithmic bytes per interior point of the GPU sweeps (each vector read or written once).
def sweep_bytes_per_point(elem_bytes: int) -> int:
    """One Chebyshev step on K: read x_k, x_{k-1}, rho; write x_{k+1}."""
    return 4 * elem_bytes


def apply_bytes_per_point(elem_bytes: int, dot_operands: int = 0) -> int:
    """One B apply: read x, write y, plus one read per fused dot operand."""
    return (2 + dot_operands) * elem_bytes


MI355X_HBM_PEAK_GBS = 8000.0
