"""The oracle against stored exact values (tests/golden/, written by
tests/golden/make_golden.py from the exact blend form)."""
import os
from fractions import Fraction

import numpy as np

from oracle import oracle

U = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))


def _load_runge():
    rows = []
    with open(os.path.join(HERE, "golden", "runge_n21_d3_exact.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t, r, lam = line.split()
            rows.append((float(t), Fraction(r), Fraction(lam)))
    return rows


def test_runge_exact_values():
    n, d = 21, 3
    nodes = (2.0 * np.arange(n) - (n - 1)) / (n - 1)
    values = 1.0 / (1.0 + 25.0 * nodes * nodes)
    rows = _load_runge()
    t = np.array([row[0] for row in rows])
    r, lam, S = oracle.evaluate(nodes, values, d, t)
    for (ti, re, le), ri, li, si in zip(rows, r, lam, S):
        # stored values carry 31 significant digits: 1e-29 relative
        assert abs(Fraction(ri) - re) <= 20 * n * U * Fraction(si) + abs(re) * Fraction(1, 10 ** 29)
        assert abs(Fraction(li) - le) <= 20 * n * U * le * (1 + le)
