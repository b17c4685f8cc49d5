"""Pins of the oracle's adjoint (dL/df_k, dL/dx_p, dL/dx_k, dL/dw_k) for the
loss L = sum_p g_p r(x_p).

References that do not share the oracle's formulas:
  * exact cardinal functions of the blend form (r is linear in f);
  * exact central differences (h = 1e-30, rational arithmetic) of the blend
    form with respect to the points and to the nodes -- the node derivative
    is the total one, the weights being recomputed from the moved nodes;
  * identities that follow from the structure of the interpolant:
    partition of unity, translation and scale invariance, invariance under a
    common weight factor, and polynomial reproduction.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, metrics, oracle
from paper_1606_06508_amd import inputs

U = 2.0 ** -53


def _loss_exact(nodes, f, d, pts, g):
    return sum((Fraction(gp) * exact.blend_eval(nodes, f, d, tp) for tp, gp in zip(pts, g)),
               Fraction(0))


@pytest.mark.parametrize("n,d", [(5, 0), (6, 2), (7, 3), (6, 5)])
def test_adjoint_matches_exact_derivatives(n, d):
    rng = np.random.default_rng(300 + 10 * n + d)
    x = inputs.equispaced(n) + rng.uniform(-0.3, 0.3, size=n) * (2.0 / (n - 1))
    assert np.all(np.diff(x) > 0)
    f = rng.standard_normal(n)
    pts = np.concatenate([rng.uniform(-1, 1, size=3), [x[2]]])  # one exact hit
    g = rng.standard_normal(pts.size)
    out = oracle.backward(x, f, d, pts, g)

    # dL/df_k = sum_p g_p b_k(x_p)
    ref_df = [Fraction(0)] * n
    for tp, gp in zip(pts, g):
        for k, bk in enumerate(exact.blend_cardinals(x, d, tp)):
            ref_df[k] += Fraction(gp) * bk
    ref_df = np.array([float(v) for v in ref_df])
    assert np.allclose(out["d_values"], ref_df, rtol=1e-12, atol=1e-13 * np.abs(ref_df).max())

    # dL/dx_p = g_p r'(x_p), also at the hit (r is smooth there)
    ref_dp = np.array([float(Fraction(gp) * exact.central_difference(
        lambda t: exact.blend_eval(x, f, d, t), tp)) for tp, gp in zip(pts, g)])
    assert np.allclose(out["d_points"], ref_dp, rtol=1e-10, atol=1e-11 * np.abs(ref_dp).max())

    # dL/dx_k total: move node k, recompute everything
    h = Fraction(1, 10 ** 30)
    xf = [Fraction(v) for v in x]
    ref_dx = []
    for k in range(n):
        xp, xm = list(xf), list(xf)
        xp[k] += h
        xm[k] -= h
        ref_dx.append(float((_loss_exact(xp, f, d, pts, g) - _loss_exact(xm, f, d, pts, g)) / (2 * h)))
    ref_dx = np.array(ref_dx)
    assert np.allclose(out["d_nodes"], ref_dx, rtol=1e-10, atol=1e-11 * np.abs(ref_dx).max())


def _medium_case(d=4, n=101, m=2000, poly=None):
    rng = np.random.default_rng(77 + d)
    x = inputs.equispaced(n)
    if poly is None:
        om, am = inputs.sines_params(rng)
        f = inputs.sines(x, om, am)
    else:
        f = np.polyval(poly, x)
    pts = np.concatenate([rng.uniform(-1, 1, size=m - 3), x[[0, 17, n - 1]]])
    g = rng.standard_normal(m)
    return x, f, pts, g


@pytest.mark.parametrize("d", [0, 3, 6])
def test_partition_of_unity(d):
    """sum_k b_k(x) = 1, so sum_k dL/df_k = sum_p g_p."""
    x, f, pts, g = _medium_case(d)
    out = oracle.backward(x, f, d, pts, g)
    assert abs(out["d_values"].sum() - g.sum()) <= 1e-12 * np.abs(g).sum()


@pytest.mark.parametrize("d", [0, 3, 6])
def test_translation_invariance(d):
    """r depends on nodes and points only through differences: moving all of
    them together changes nothing, so the node and point gradients cancel."""
    x, f, pts, g = _medium_case(d)
    out = oracle.backward(x, f, d, pts, g)
    tot = out["d_nodes"].sum() + out["d_points"].sum()
    scale = np.abs(out["d_nodes"]).sum() + np.abs(out["d_points"]).sum()
    assert abs(tot) <= 1e-11 * scale


@pytest.mark.parametrize("d", [0, 3, 6])
def test_scale_invariance(d):
    """Weights are homogeneous in the node differences, so r(c x; c nodes) =
    r(x; nodes): sum x_k dL/dx_k + sum x_p dL/dx_p = 0."""
    x, f, pts, g = _medium_case(d)
    out = oracle.backward(x, f, d, pts, g)
    tot = (x * out["d_nodes"]).sum() + (pts * out["d_points"]).sum()
    scale = np.abs(x * out["d_nodes"]).sum() + np.abs(pts * out["d_points"]).sum()
    assert abs(tot) <= 1e-11 * scale


@pytest.mark.parametrize("d", [1, 4])
def test_common_weight_factor_invariance(d):
    """r is unchanged when every weight is multiplied by the same factor, so
    sum_k w_k dL/dw_k = 0."""
    x, f, pts, g = _medium_case(d)
    out = oracle.backward(x, f, d, pts, g)
    w = oracle.weights(x, d)
    assert abs((w * out["d_weights"]).sum()) <= 1e-11 * np.abs(w * out["d_weights"]).sum()


@pytest.mark.parametrize("d", [2, 5])
def test_polynomial_data_gradients(d):
    """For data from p of degree <= d, r = p whatever the nodes, as long as each
    value moves with its node (f_k = p(x_k)).  Hence dL/dx_p = g_p p'(x_p) and
    dL/dx_k + p'(x_k) dL/df_k = 0 for every node."""
    rng = np.random.default_rng(9)
    poly = rng.standard_normal(d + 1)
    x, f, pts, g = _medium_case(d, poly=poly)
    out = oracle.backward(x, f, d, pts, g)
    dp_ref = g * np.polyval(np.polyder(poly), pts)
    assert np.allclose(out["d_points"], dp_ref, rtol=1e-9, atol=1e-9 * np.abs(dp_ref).max())
    moved = out["d_nodes"] + np.polyval(np.polyder(poly), x) * out["d_values"]
    scale = np.abs(out["d_nodes"]).sum() + np.abs(np.polyval(np.polyder(poly), x) * out["d_values"]).sum()
    assert np.abs(moved).max() <= 1e-11 * scale


def test_linear_in_values():
    """r is linear in f: a finite difference in f with a large step is exact
    up to rounding."""
    x, f, pts, g = _medium_case(3, n=41, m=300)
    out = oracle.backward(x, f, 3, pts, g)
    for k in (0, 7, 20, 40):
        e = np.zeros_like(f)
        e[k] = 1.0
        lp = g @ oracle.evaluate(x, f + e, 3, pts, lebesgue=False, scale=False)[0]
        lm = g @ oracle.evaluate(x, f - e, 3, pts, lebesgue=False, scale=False)[0]
        assert abs((lp - lm) / 2 - out["d_values"][k]) <= 1e-12 * np.abs(g).sum() * 10


def test_central_differences_double():
    """Central differences (h = 1e-6) of the binary64 forward pass agree with the
    adjoint within the truncation-plus-rounding error model of the difference:
    10 (h^2 M3 / 6 + 2 u sum|g r| / h), M3 estimated from differences at 10h."""
    n, d, m = 65, 4, 400
    rng = np.random.default_rng(5)
    x = inputs.equispaced(n)
    om, am = inputs.sines_params(rng)
    f = inputs.sines(x, om, am)
    pts = rng.uniform(-1, 1, size=m)
    g = rng.standard_normal(m)
    out = oracle.backward(x, f, d, pts, g)
    r0 = oracle.evaluate(x, f, d, pts, lebesgue=False, scale=False)[0]
    noise = 2 * U * np.abs(g * r0).sum()
    h = 1e-6

    def L(nodes):
        return g @ oracle.evaluate(nodes, f, d, pts, lebesgue=False, scale=False)[0]

    for k in (0, 1, 16, 32, 63, 64):
        def fd(step):
            xp, xm = x.copy(), x.copy()
            xp[k] += step
            xm[k] -= step
            return (L(xp) - L(xm)) / (2 * step)
        a, b = fd(h), fd(10 * h)
        m3 = abs(b - a) * 6 / (99 * h * h) if b != a else 0.0
        tol = 10 * (h * h * m3 / 6 + noise / h)
        assert abs(a - out["d_nodes"][k]) <= tol, (k, a, out["d_nodes"][k], tol)


@pytest.mark.parametrize("n,d", [(1, 0), (2, 1), (33, 3), (257, 4)])
def test_grad_scales_c_matches_numpy(n, d):
    """The C error scales of the adjoint (fho_grad_scales, used at full
    sizes) against the independent numpy sums (metrics.grad_scales plus the
    dense weight-derivative matrix), with hits and a NaN point.  The two
    weight each point by 1 + Lambda from differently rounded sums of
    D (plain here, compensated in the numpy path), which differ by about
    u Lambda at extrapolated points: rtol 1e-6 for a tolerance scale."""
    rng = np.random.default_rng(40 + n)
    x = inputs.equispaced(n) if n > 1 else np.array([0.25])
    f = rng.standard_normal(n)
    pts = np.concatenate([rng.uniform(-1.2, 1.2, 500), x[:: max(1, n // 4)], [np.nan]])
    g = rng.standard_normal(pts.size)
    s_df, s_dx, s_dxd, s_dw = metrics.grad_scales(x, f, d, pts, g)
    s_dn = s_dxd + metrics.weight_derivative_abs(x, d).T @ s_dw
    c_df, c_dx, c_dn = oracle.grad_scales(x, f, d, pts, g)
    for a, b in ((s_df, c_df), (s_dx, c_dx), (s_dn, c_dn)):
        assert np.allclose(a, b, rtol=1e-6, atol=0.0)
