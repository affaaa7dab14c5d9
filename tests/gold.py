"""Reader of the stored oracle samples under tests/golden/ (written by
tests/golden/make_oracle_samples.py, which calls only the oracle)."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def samples(fname):
    """(node indices, oracle values, max |u| over fluid nodes) of one stored sample file."""
    path = os.path.join(GOLD, fname)
    if not os.path.exists(path):
        pytest.skip(f"{fname} not generated")
    data = np.loadtxt(path, comments="#")
    umax = None
    for line in open(path):
        if line.startswith("# max_abs_u_fluid"):
            umax = float(line.split()[-1])
    return data[:, 0].astype(np.int64), data[:, 1], umax
