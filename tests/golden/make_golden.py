"""Writes tests/golden/runge_n21_d3_exact.txt: exact values (rational arithmetic,
printed to 30 significant digits) of the Floater-Hormann interpolant and its
Lebesgue function for the Runge data on 21 equispaced nodes with d = 3.

The values come from the blend definition of the interpolant (Floater &
Hormann 2007), evaluated exactly by oracle/exact.py; nothing here calls the
binary64 oracle or the GPU library.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import exact  # noqa: E402

getcontext().prec = 40


def dec(q: Fraction) -> str:
    return "{:.30e}".format(Decimal(q.numerator) / Decimal(q.denominator))


def main():
    n, d = 21, 3
    nodes = [(2.0 * k - (n - 1)) / (n - 1) for k in range(n)]
    values = [1.0 / (1.0 + 25.0 * x * x) for x in nodes]
    pts = [k / 64.0 for k in range(-64, 65, 9)] + [0.123456789, -0.987654321, 0.3, -0.05, 0.95]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "runge_n21_d3_exact.txt")
    with open(out, "w") as fh:
        fh.write("# Floater-Hormann interpolant of f(x)=1/(1+25x^2) on 21 equispaced nodes\n")
        fh.write("# x_k=(2k-20)/20 (binary64), f_k = binary64 1/(1+25 x_k^2), d=3.\n")
        fh.write("# Exact rational values from the blend form (Floater & Hormann 2007),\n")
        fh.write("# written by tests/golden/make_golden.py.  Columns: t  r(t)  Lambda(t)\n")
        for t in pts:
            r = exact.blend_eval(nodes, values, d, t)
            lam = exact.blend_lebesgue(nodes, d, t)
            fh.write("{!r} {} {}\n".format(t, dec(r), dec(lam)))
    print("wrote", out)


if __name__ == "__main__":
    main()
