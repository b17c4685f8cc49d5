"""Exact rational Floater-Hormann interpolation, used to pin the FP64 oracle.

TEST INFRASTRUCTURE ONLY (imported by the test-suite and by the script that
writes the golden fixtures; never by the product package).

This module deliberately does NOT use the barycentric (second) form or the
weight formula that the oracle and the kernels evaluate.  It evaluates the
interpolant through its *blend* definition (Floater & Hormann, Numer. Math.
107, 2007: the construction of r as a blend of local interpolating
polynomials):

    r(x) = sum_{i=0}^{n-1-d} lambda_i(x) p_i(x) / sum_{i=0}^{n-1-d} lambda_i(x),
    lambda_i(x) = (-1)^i / prod_{j=i}^{i+d} (x - x_j),

where p_i is the polynomial of degree <= d interpolating f at x_i..x_{i+d}
(evaluated here in Lagrange form).  In exact arithmetic this equals the
barycentric form, so agreement between the two is a genuine check of the
weights, the sign convention and the second-form sum.  Everything here is
exact (fractions.Fraction); binary64 inputs convert exactly.

Also provided: classical Lagrange interpolation (the d = n-1 special case),
the cardinal functions b_k of the blend (for the Lebesgue function
sum_k |b_k|), and exact central differences for derivative checks.
"""
from fractions import Fraction
from typing import List, Sequence

Frac = Fraction


def F(v) -> Fraction:
    """Exact rational value of a float / int / Fraction."""
    if isinstance(v, Fraction):
        return v
    return Fraction(v)


def _lagrange_basis(xs: Sequence[Fraction], t: Fraction) -> List[Fraction]:
    """l_j(t) for the polynomial interpolant on the nodes xs (t not a node)."""
    out = []
    for j, xj in enumerate(xs):
        num = Fraction(1)
        den = Fraction(1)
        for l, xl in enumerate(xs):
            if l != j:
                num *= t - xl
                den *= xj - xl
        out.append(num / den)
    return out


def lagrange_eval(nodes, values, t) -> Fraction:
    """Polynomial interpolant of (nodes, values) at t, exact."""
    xs = [F(v) for v in nodes]
    fs = [F(v) for v in values]
    t = F(t)
    for j, xj in enumerate(xs):
        if t == xj:
            return fs[j]
    return sum((b * f for b, f in zip(_lagrange_basis(xs, t), fs)), Fraction(0))


def lagrange_lebesgue(nodes, t) -> Fraction:
    """Lebesgue function sum_k |l_k(t)| of polynomial interpolation."""
    xs = [F(v) for v in nodes]
    t = F(t)
    if any(t == xj for xj in xs):
        return Fraction(1)
    return sum((abs(b) for b in _lagrange_basis(xs, t)), Fraction(0))


def blend_cardinals(nodes, d: int, t) -> List[Fraction]:
    """Cardinal functions b_k(t) of the FH blend: r(t) = sum_k b_k(t) f_k."""
    xs = [F(v) for v in nodes]
    n = len(xs)
    t = F(t)
    for j, xj in enumerate(xs):
        if t == xj:
            return [Fraction(1) if k == j else Fraction(0) for k in range(n)]
    b = [Fraction(0)] * n
    lam_sum = Fraction(0)
    for i in range(n - d):
        prod = Fraction(1)
        for j in range(i, i + d + 1):
            prod *= t - xs[j]
        lam = Fraction((-1) ** i) / prod
        lam_sum += lam
        basis = _lagrange_basis(xs[i:i + d + 1], t)
        for jj, bj in enumerate(basis):
            b[i + jj] += lam * bj
    return [bk / lam_sum for bk in b]


def blend_eval(nodes, values, d: int, t) -> Fraction:
    """FH interpolant at t via the blend of local polynomials, exact."""
    fs = [F(v) for v in values]
    return sum((bk * fk for bk, fk in zip(blend_cardinals(nodes, d, t), fs)), Fraction(0))


def blend_lebesgue(nodes, d: int, t) -> Fraction:
    """FH Lebesgue function sum_k |b_k(t)|, exact."""
    return sum((abs(bk) for bk in blend_cardinals(nodes, d, t)), Fraction(0))


def central_difference(fun, t, h=Fraction(1, 10 ** 30)) -> Fraction:
    """(fun(t+h) - fun(t-h)) / 2h in exact arithmetic.

    For a rational function smooth near t the truncation error is
    O(h^2 |fun'''|), i.e. far below binary64 resolution for h = 1e-30.
    """
    t = F(t)
    return (fun(t + h) - fun(t - h)) / (2 * h)


def to_float(q: Fraction) -> float:
    """Correctly rounded binary64 value of an exact rational."""
    return float(q)


def cardinal_derivatives(nodes, d: int, t, h=Fraction(1, 10 ** 30)) -> List[Fraction]:
    """b_k'(t) of the blend cardinals by exact central differences (also at a
    node, where the cardinals are smooth; truncation O(h^2))."""
    t = F(t)
    bp = blend_cardinals(nodes, d, t + h)
    bm = blend_cardinals(nodes, d, t - h)
    return [(p - m) / (2 * h) for p, m in zip(bp, bm)]


EPS = Fraction(1, 2 ** 100)


def term_sensitivities(fun, groups, eps=EPS):
    """First-order worst-case sensitivity of a computation to relative
    errors in its terms, by experiment: `groups` is a list of lists of exact
    terms, `fun(groups)` returns the result (a Fraction or a list of them).
    Every term is perturbed alone by the relative amount eps and the changes
    of the result are added in absolute value (per component for a list):
    sum over terms of |fun(term * (1 + eps)) - fun()| / eps.  No formula for
    the sensitivity is used; for eps -> 0 this is sum |d fun / d term * term|,
    the largest first-order change when every term carries its own relative
    error of at most one unit."""
    base = fun(groups)
    single = not isinstance(base, list)
    base_l = [base] if single else base
    tot = [Fraction(0)] * len(base_l)
    for gi, grp in enumerate(groups):
        for k, v in enumerate(grp):
            if v == 0:
                continue
            pert = list(groups)
            pert[gi] = list(grp)
            pert[gi][k] = v * (1 + eps)
            out = fun(pert)
            out_l = [out] if single else out
            for c, (o, b) in enumerate(zip(out_l, base_l)):
                tot[c] += abs(o - b)
    res = [s / eps for s in tot]
    return res[0] if single else res
