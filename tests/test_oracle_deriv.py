"""Pins of the oracle's derivative r'(x) (fho_eval_deriv) to facts that do
not come from the oracle:

- exact-rational central differences (h = 1e-30) of the blend form
  sum lambda_i p_i / sum lambda_i, a different algorithm reaching the same
  function, at random points and across the nodes (where the oracle uses
  the node formula of Schneider and Werner);
- polynomials of degree <= d are reproduced, so r' = p' up to rounding;
- the derivative equals the adjoint's dL/dx_p for L = sum_p r(x_p);
- NaN and infinite points give NaN.
Tolerances are multiples of u times the oracle's own error scale S'.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, oracle
from paper_1606_06508_amd import inputs

U = 2.0 ** -53


@pytest.mark.parametrize("n,d", [(2, 1), (5, 0), (6, 2), (9, 3), (12, 5), (12, 11)])
def test_against_exact_blend_form(n, d):
    g = np.random.default_rng(300 + 10 * n + d)
    nodes = np.sort(inputs.equispaced(n) + (g.uniform(-0.2, 0.2, n) * 2.0 / (n - 1) if n > 2 else 0))
    vals = g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1.0, 1.0, 25), [1.3, -1.25]])
    r, dr, sc = oracle.eval_deriv(nodes, vals, d, pts)
    for i, t in enumerate(pts):
        want = float(exact.central_difference(lambda s: exact.blend_eval(nodes, vals, d, s), t))
        assert abs(dr[i] - want) <= 20 * n * U * sc[i], (i, t, dr[i], want)


@pytest.mark.parametrize("n,d", [(3, 1), (7, 2), (10, 4), (8, 7)])
def test_node_formula_against_exact_limit(n, d):
    """At a node the oracle takes r'(x_j) from the node formula; the exact
    blend form differenced across the node gives the same number."""
    g = np.random.default_rng(400 + n + d)
    nodes = np.sort(inputs.equispaced(n) + g.uniform(-0.1, 0.1, n) * 2.0 / (n - 1))
    vals = g.standard_normal(n)
    r, dr, sc = oracle.eval_deriv(nodes, vals, d, nodes)
    assert np.array_equal(r, vals)
    for j in range(n):
        want = float(exact.central_difference(lambda s: exact.blend_eval(nodes, vals, d, s),
                                              Fraction(nodes[j])))
        assert abs(dr[j] - want) <= 20 * n * U * sc[j] + 1e-300, (j, dr[j], want)


@pytest.mark.parametrize("d", [0, 1, 3, 6])
def test_polynomial_reproduction(d):
    g = np.random.default_rng(d)
    nodes = inputs.equispaced(41)
    coef = g.standard_normal(d + 1)
    vals = np.polyval(coef, nodes)
    pts = np.concatenate([g.uniform(-1, 1, 400), nodes[::5]])
    r, dr, sc = oracle.eval_deriv(nodes, vals, d, pts)
    want = np.polyval(np.polyder(coef), pts) if d > 0 else np.zeros_like(pts)
    assert np.all(np.abs(dr - want) <= 50 * U * sc + 1e-300)


def test_matches_adjoint_point_gradient():
    c = inputs.grad_workload(n=129, m=2000)
    r, dr, sc = oracle.eval_deriv(c["nodes"], c["values"], c["d"], c["points"])
    o = oracle.backward(c["nodes"], c["values"], c["d"], c["points"], np.ones(c["points"].size))
    assert np.all(np.abs(dr - o["d_points"]) <= 1e-13 * sc)


def test_non_finite_points_and_given_weights():
    nodes = inputs.equispaced(9)
    vals = np.sin(3 * nodes)
    pts = np.array([np.nan, np.inf, -np.inf, 0.1])
    r, dr, _ = oracle.eval_deriv(nodes, vals, 2, pts)
    assert np.all(np.isnan(r[:3])) and np.all(np.isnan(dr[:3])) and np.isfinite(dr[3])
    # weights passed in (scaled by a power of two) give the same bits
    w = oracle.weights(nodes, 2)
    r2, dr2, _ = oracle.eval_deriv(nodes, vals, 2, pts[3:], w=np.ldexp(w, 7))
    assert r2[0] == r[3] and dr2[0] == dr[3]
