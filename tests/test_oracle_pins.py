"""Pins of the FP64 oracle against facts fixed by the mathematics of
Floater-Hormann interpolation (not against the oracle's own formula).

Each test names the fact it checks.  A plausible slip in the oracle (a
dropped term, a wrong sign or index in the weights, a transposed quotient,
a mishandled hit) fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, oracle
from paper_1606_06508_amd import inputs

U = 2.0 ** -53


def _nodes_random(n, g, lo=-1.0, hi=1.0):
    x = np.sort(g.uniform(lo, hi, size=n))
    assert np.all(np.diff(x) > 0)
    return x


def _econd(r_hat, r_ref, S):
    return np.abs(r_hat - r_ref) / S


# ---------------------------------------------------------------- P1 / P5 --
@pytest.mark.parametrize("d", [0, 1, 3, 8, 36])
def test_interpolates_nodes_bitwise(d):
    """r(x_k) = f_k exactly and Lambda(x_k) = 1 (FH interpolates its data)."""
    g = np.random.default_rng(1)
    x = _nodes_random(37, g)
    f = g.standard_normal(37)
    r, lam, _ = oracle.evaluate(x, f, d, x)
    assert np.array_equal(r.view(np.int64), f.view(np.int64))
    assert np.all(lam == 1.0)


@pytest.mark.parametrize("d", [0, 2, 5, 10])
def test_lebesgue_at_least_one(d):
    """Lambda = sum|b_k| >= |sum b_k| = 1 everywhere (partition of unity)."""
    g = np.random.default_rng(2)
    x = inputs.cheb2(41) if d % 2 else inputs.equispaced(41)
    t = g.uniform(-1.2, 1.2, size=4000)
    _, lam, _ = oracle.evaluate(x, np.zeros(41), d, t)
    assert np.all(lam >= 1.0 - 4 * U)


# --------------------------------------------------------------------- P2 --
@pytest.mark.parametrize("d", [0, 1, 2, 4, 7])
def test_reproduces_polynomials_of_degree_d(d):
    """FH reproduces every polynomial of degree <= d.  Integer nodes and
    integer coefficients make the data exact, so the only error is the
    evaluation's own, bounded by a few u times S."""
    g = np.random.default_rng(10 + d)
    n = 40
    x = np.arange(n, dtype=np.float64)
    c = g.integers(-3, 4, size=d + 1)
    f = np.array([sum(int(c[j]) * int(k) ** j for j in range(d + 1)) for k in range(n)],
                 dtype=np.float64)
    assert np.all(np.abs(f) < 2 ** 53)
    t = g.uniform(-0.5, n - 0.5, size=300)
    r, _, S = oracle.evaluate(x, f, d, t)
    for ti, ri, si in zip(t, r, S):
        exact_p = sum(int(c[j]) * Fraction(ti) ** j for j in range(d + 1))
        assert abs(Fraction(ri) - exact_p) <= 50 * U * Fraction(si)


# --------------------------------------------------------------------- P3 --
@pytest.mark.parametrize("n", [2, 3, 5, 8, 10])
def test_full_degree_is_lagrange(n):
    """d = n-1 is polynomial interpolation (one blend window)."""
    g = np.random.default_rng(20 + n)
    x = _nodes_random(n, g)
    f = g.standard_normal(n)
    t = g.uniform(-1.1, 1.1, size=40)
    r, lam, S = oracle.evaluate(x, f, n - 1, t)
    for ti, ri, li, si in zip(t, r, lam, S):
        assert abs(Fraction(ri) - exact.lagrange_eval(x, f, ti)) <= 20 * n * U * Fraction(si)
        le = exact.lagrange_lebesgue(x, ti)
        # D = sum a_k has condition number Lambda, so Lambda's own relative
        # error is of order u (1 + Lambda).
        assert abs(Fraction(li) - le) <= 20 * n * U * le * (1 + le)


# --------------------------------------------------------------------- P4 --
def test_berrut_weights_at_degree_zero():
    """d = 0: every J_k = {k} and the product is empty, so w_k = (-1)^k exactly
    for any nodes."""
    g = np.random.default_rng(4)
    for n in (1, 2, 7, 100):
        x = _nodes_random(n, g, -50, 50)
        w = oracle.weights(x, 0)
        assert np.array_equal(w, np.array([(-1.0) ** k for k in range(n)]))


# --------------------------------------------------------------------- P6 --
@pytest.mark.parametrize("d", [0, 1, 2, 3, 4, 5, 6])
def test_equispaced_closed_form(d):
    """On x_k = k (spacing 1): |w_k| d! = sum_{i in J_k} C(d, k-i) and the sign
    alternates as (-1)^(k-d)."""
    n = 30
    x = np.arange(n, dtype=np.float64)
    w = oracle.weights(x, d)
    for k in range(n):
        lo, hi = max(0, k - d), min(k, n - 1 - d)
        target = sum(math.comb(d, k - i) for i in range(lo, hi + 1))
        got = abs(w[k]) * math.factorial(d)
        if d <= 2:
            assert got == target
        else:
            assert abs(got - target) <= 4 * (d + 1) * U * target
        assert math.copysign(1.0, w[k]) == (-1.0) ** (k - d)


def test_equispaced_small_degree_pattern():
    """The familiar patterns 1,1,..; 1,2,..,2,1; 1,3,4,..,4,3,1; 1,4,7,8,..,8,7,4,1."""
    n = 12
    x = np.arange(n, dtype=np.float64)
    pats = {0: [1] * n, 1: [1] + [2] * (n - 2) + [1],
            2: [1, 3] + [4] * (n - 4) + [3, 1], 3: [1, 4, 7] + [8] * (n - 6) + [7, 4, 1]}
    for d, p in pats.items():
        w = np.abs(oracle.weights(x, d)) * math.factorial(d)
        assert np.allclose(w, p, rtol=8 * U * 4, atol=0)


# --------------------------------------------------------------------- P7 --
def test_full_degree_weights_are_classical():
    """d = n-1: w_k = prod_{j != k} 1/(x_k - x_j) (classical barycentric weights)."""
    g = np.random.default_rng(7)
    for n in (2, 5, 9, 14):
        x = _nodes_random(n, g)
        w = oracle.weights(x, n - 1)
        for k in range(n):
            ref = Fraction(1)
            for j in range(n):
                if j != k:
                    ref /= Fraction(x[k]) - Fraction(x[j])
            assert abs(Fraction(w[k]) - ref) <= 2 * n * U * abs(ref)


# --------------------------------------------------------------------- P8 --
@pytest.mark.parametrize("d", [0, 1, 3, 6])
def test_constants_are_reproduced(d):
    g = np.random.default_rng(8)
    x = inputs.cheb2(33)
    f = np.full(33, -2.75)
    t = g.uniform(-1, 1, size=2000)
    r, _, S = oracle.evaluate(x, f, d, t)
    assert np.all(_econd(r, -2.75, S) <= 50 * U)


# --------------------------------------------------------------------- P9 --
@pytest.mark.parametrize("e", [-300, -37, 1, 52, 400])
def test_power_of_two_weight_scaling_is_invisible(e):
    """Scaling every weight by 2^e is exact (the paper's fact (rndA): a power of
    two times a normal number is exact when the result stays normal), so every
    a_k scales exactly and r, Lambda are unchanged bit-for-bit."""
    c = inputs.runge()
    w = oracle.weights(c["nodes"], c["d"])
    ws = np.ldexp(w, e)
    assert np.all(np.isfinite(ws)) and np.all(np.abs(ws) >= np.finfo(float).tiny * 2 ** 60)
    r0, l0, _ = oracle.evaluate(c["nodes"], c["values"], c["d"], c["points"], w=w)
    r1, l1, _ = oracle.evaluate(c["nodes"], c["values"], c["d"], c["points"], w=ws)
    assert np.array_equal(r0, r1) and np.array_equal(l0, l1)


# -------------------------------------------------------------------- P10 --
@pytest.mark.parametrize("d", [1, 2, 5])
def test_symmetric_nodes(d):
    """x_{n-1-k} = -x_k gives |w_{n-1-k}| = |w_k|, Lambda(-t) = Lambda(t), and
    r(-t) = r(t) for even data."""
    n = 51
    x = inputs.equispaced(n)
    assert np.array_equal(x[::-1], -x)
    w = oracle.weights(x, d)
    assert np.all(np.abs(np.abs(w[::-1]) - np.abs(w)) <= 4 * (d + 1) * U * np.abs(w))
    f = np.cos(3 * np.abs(x))
    g = np.random.default_rng(10)
    t = g.uniform(-1, 1, size=1000)
    r1, l1, s1 = oracle.evaluate(x, f, d, t)
    r2, l2, s2 = oracle.evaluate(x, f, d, -t)
    assert np.all(np.abs(r1 - r2) <= 50 * U * np.maximum(s1, s2))
    assert np.all(np.abs(l1 - l2) <= 50 * U * l1)


# -------------------------------------------------------------------- P12 --
@pytest.mark.parametrize("n,d", [(4, 0), (4, 2), (7, 1), (7, 3), (9, 4), (12, 2), (12, 6),
                                 (12, 11)])
def test_second_form_equals_blend(n, d):
    """Barycentric form with FH weights == the blend sum lambda_i p_i / sum lambda_i,
    evaluated exactly: this pins the weight formula, its sign and the sum."""
    g = np.random.default_rng(100 * n + d)
    x = _nodes_random(n, g)
    f = g.standard_normal(n)
    t = np.concatenate([g.uniform(-1.3, 1.3, size=12), x[:2]])
    r, lam, S = oracle.evaluate(x, f, d, t)
    for ti, ri, li, si in zip(t, r, lam, S):
        rb = exact.blend_eval(x, f, d, ti)
        lb = exact.blend_lebesgue(x, d, ti)
        assert abs(Fraction(ri) - rb) <= 20 * n * U * Fraction(si), (ti, ri, float(rb))
        assert abs(Fraction(li) - lb) <= 20 * n * U * lb * (1 + lb)


def test_second_form_equals_blend_larger_n():
    g = np.random.default_rng(55)
    n, d = 64, 5
    x = inputs.cheb2(n)
    f = g.standard_normal(n)
    t = g.uniform(-1, 1, size=4)
    r, lam, S = oracle.evaluate(x, f, d, t)
    for ti, ri, li, si in zip(t, r, lam, S):
        assert abs(Fraction(ri) - exact.blend_eval(x, f, d, ti)) <= 4 * U * Fraction(si)
        lb = exact.blend_lebesgue(x, d, ti)
        assert abs(Fraction(li) - lb) <= 4 * U * lb * (1 + lb)


# ----------------------------------------------------------- conventions --
def test_nan_and_inf_points():
    c = inputs.runge()
    t = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0])
    r, lam, _ = oracle.evaluate(c["nodes"], c["values"], 3, t)
    assert np.isnan(r[0]) and np.isnan(lam[0])
    assert np.isnan(r[1]) and np.isnan(r[2])          # all a_k = 0, 0/0
    j = int(np.flatnonzero(c["nodes"] == 0.0)[0])      # 0.0 is node 10 of 21
    assert r[3] == c["values"][j] and r[4] == c["values"][j] and lam[3] == lam[4] == 1.0


def test_nan_value_poisons_all_but_other_hits():
    c = inputs.runge()
    f = c["values"].copy()
    f[4] = np.nan
    t = np.concatenate([[0.123, -0.77], c["nodes"]])
    r, _, _ = oracle.evaluate(c["nodes"], f, 3, t)
    assert np.isnan(r[0]) and np.isnan(r[1])
    assert np.isnan(r[2 + 4])
    others = np.delete(np.arange(21), 4)
    assert np.array_equal(r[2 + others], f[others])


@pytest.mark.parametrize("nodes,d,code", [
    ([], 0, 1), ([0.0, 1.0], -1, 2), ([0.0, 1.0], 2, 2), ([0.0, 0.0, 1.0], 1, 3),
    ([1.0, 0.0], 0, 3), ([0.0, np.nan], 0, 4), ([0.0, np.inf], 1, 4)])
def test_error_codes(nodes, d, code):
    with pytest.raises(oracle.OracleError) as e:
        oracle.weights(np.array(nodes, dtype=float), d)
    assert e.value.code == code


def test_thread_count_does_not_change_results():
    c = inputs.sines_workload(n=301, m=5000)
    a = oracle.evaluate(c["nodes"], c["values"], 4, c["points"], nthreads=1)
    b = oracle.evaluate(c["nodes"], c["values"], 4, c["points"], nthreads=7)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_compensation_is_at_least_as_accurate():
    """The compensated oracle is closer to the exact value than the plain sum
    on average (it must be the more accurate side of every comparison)."""
    g = np.random.default_rng(3)
    n, d = 12, 3
    x = _nodes_random(n, g)
    f = g.standard_normal(n) * 1e3 + 1e4
    t = g.uniform(-1, 1, size=60)
    rc, _, _ = oracle.evaluate(x, f, d, t, compensated=True)
    rp, _, _ = oracle.evaluate(x, f, d, t, compensated=False)
    ec = ep = 0.0
    for ti, a, b in zip(t, rc, rp):
        ex = exact.blend_eval(x, f, d, ti)
        ec += float(abs(Fraction(a) - ex))
        ep += float(abs(Fraction(b) - ex))
    assert ec <= ep


# ------------------------------------------------------------------- P11 --
@pytest.mark.parametrize("d", [3, 8])
def test_oracle_own_error_against_sixty_digit_evaluation(d):
    """The oracle's rounding error on the 1001-node sines workload, against
    the same second form (same binary64 weights, values and points) summed
    in 60-digit decimal arithmetic: e_cond(r) <= 4u and
    |Lambda - Lambda_ref| <= 4u Lambda (1 + Lambda)."""
    from decimal import Decimal, localcontext

    c = inputs.sines_workload(m=150)
    nodes, vals, pts = c["nodes"], c["values"], c["points"]
    w = oracle.weights(nodes, d)
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    xs = [Decimal(float(v)) for v in nodes]
    ws = [Decimal(float(v)) for v in w]
    fs = [Decimal(float(v)) for v in vals]
    with localcontext() as ctx:
        ctx.prec = 60
        for p, t in enumerate(pts):
            td = Decimal(float(t))
            N = D = L = Decimal(0)
            for xk, wk, fk in zip(xs, ws, fs):
                a = wk / (td - xk)
                N += a * fk
                D += a
                L += abs(a)
            r_ref, lam_ref = float(N / D), float(L / abs(D))
            assert abs(r_o[p] - r_ref) <= 4 * U * s_o[p], (p, r_o[p], r_ref)
            assert abs(lam_o[p] - lam_ref) <= 4 * U * lam_ref * (1 + lam_ref), p


@pytest.mark.parametrize("family", ["equispaced", "cheb2", "jittered", "random"])
def test_weights_alternate_strictly_in_sign(family):
    """Floater-Hormann weights alternate strictly in sign: every term of the
    sum that defines w_k has the sign (-1)^(k-d) (the no-poles argument of
    Floater & Hormann 2007), so w_k w_{k+1} < 0 for every k.  The block sums
    of the evaluation kernels rely on it.  Checked on the oracle's weights
    for random node sets, n = 2..120 and every degree up to 10 (and in exact
    rationals on a small set)."""
    g = np.random.default_rng({"equispaced": 1, "cheb2": 2, "jittered": 3, "random": 4}[family])
    for n in list(range(2, 20)) + [37, 64, 120]:
        if family == "equispaced":
            nodes = inputs.equispaced(n)
        elif family == "cheb2":
            nodes = inputs.cheb2(n)
        elif family == "jittered":
            nodes = inputs.jittered_nodes(n, g, rel=0.3) if n > 2 else inputs.equispaced(n)
        else:  # gaps spanning six orders of magnitude
            nodes = np.cumsum(10.0 ** g.uniform(-6, 0, n))
        for d in range(0, min(n - 1, 10) + 1):
            w = oracle.weights(nodes, d)
            assert np.all(w[:-1] * w[1:] < 0), (n, d)
            assert np.all(np.sign(w) == (-1.0) ** (np.arange(n) - d)), (n, d)
    # exact rationals: the sign pattern is a property of the formula, not of rounding
    xs = [Fraction(0), Fraction(1, 7), Fraction(1, 3), Fraction(1, 2), Fraction(5, 6), Fraction(1)]
    for d in range(len(xs)):
        for k in range(len(xs)):
            terms = []
            for i in range(max(0, k - d), min(k, len(xs) - 1 - d) + 1):
                prod = Fraction(1)
                for j in range(i, i + d + 1):
                    if j != k:
                        prod *= xs[k] - xs[j]
                terms.append(Fraction((-1) ** i) / prod)
            assert all((t > 0) == ((k - d) % 2 == 0) for t in terms), (d, k)
