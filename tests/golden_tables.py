"""Readers of the paper's printed tables kept as text fixtures in tests/golden/."""

import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table(name):
    """Rows of a fixture as a float array (comment lines start with #)."""
    rows = []
    for line in open(os.path.join(HERE, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return np.array(rows)
