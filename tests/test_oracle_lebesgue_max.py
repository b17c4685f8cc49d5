"""Pins of the oracle's Lebesgue-constant search (fho_lebesgue_max) to facts
that do not come from the oracle:

- polynomial interpolation (d = n - 1): on each interval the Lebesgue
  function is the polynomial sum_j s_j l_j(x) (the signs s_j of the
  Lagrange basis are constant between nodes), so its maximum is found from
  the real roots of the derivative (numpy's polynomial routines); three
  equispaced nodes give 5/4 at +-1/2 in closed form;
- FH with d < n - 1: golden-section search on the exact-rational Lebesgue
  function of the blend form sum |b_k(x)| (a different formula and a
  different search) lands on the same maxima;
- two nodes: linear interpolation, Lambda = 1 on the interval;
- power-of-two scaling of the nodes leaves every maximum bit-for-bit
  unchanged and scales every location exactly (fact rndA of the paper's
  proofs appendix);
- symmetric nodes give mirrored maxima; more rounds never lower a maximum;
  no point of a dense random sample exceeds the maximum found.
"""
from fractions import Fraction

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle import exact, oracle
from paper_1606_06508_amd import inputs

U = 2.0 ** -53


def _poly_lebesgue_maxima(nodes):
    """Per-interval maxima (value, location) of sum_j |l_j| from the roots of
    the derivative of the interval's polynomial."""
    n = nodes.size
    basis = []
    for j in range(n):
        others = np.delete(nodes, j)
        basis.append(P.polyfromroots(others) / np.prod(nodes[j] - others))
    out = []
    for k in range(n - 1):
        a, b = nodes[k], nodes[k + 1]
        mid = 0.5 * (a + b)
        lam = sum(np.sign(P.polyval(mid, c)) * c for c in basis)
        crit = [r.real for r in P.polyroots(P.polyder(lam)) if abs(r.imag) < 1e-9 and a < r.real < b]
        # values at the critical points in exact arithmetic (the monomial
        # form loses digits when Lambda is large)
        cand = [(float(exact.lagrange_lebesgue(nodes, Fraction(float(t)))), t) for t in crit]
        out.append(max(cand + [(1.0, a), (1.0, b)]))
    return out


def _tol(v):
    """Every evaluation of Lambda carries a relative error of order u Lambda
    (the rounding of each term a_k; the conditioning limit of the parity
    bars), the oracle's included."""
    return (1e-13 + 8 * U * v) * v


def _node_sets(n):
    g = np.random.default_rng(77 + n)
    rnd = np.sort(g.uniform(-1, 1, n))
    rnd[0], rnd[-1] = -1.0, 1.0
    return {"equispaced": inputs.equispaced(n), "cheb2": inputs.cheb2(n), "random": rnd}


@pytest.mark.parametrize("n", [3, 4, 5, 7, 9])
def test_polynomial_case_against_derivative_roots(n):
    for name, nodes in _node_sets(n).items():
        lam, loc, (best, at) = oracle.lebesgue_max(nodes, n - 1, samples=64, rounds=6)
        want = _poly_lebesgue_maxima(nodes)
        for k, (v, t) in enumerate(want):
            width = nodes[k + 1] - nodes[k]
            assert abs(lam[k] - v) <= _tol(v), (name, k, lam[k], v)
            assert abs(loc[k] - t) <= 1e-6 * width, (name, k, loc[k], t)
        assert best == max(lam) and at == loc[int(np.argmax(lam))]


def test_three_equispaced_nodes_closed_form():
    """l_0 + l_1 + l_2 with signs on [0, 1] is 1 + x - x^2: maximum 5/4 at 1/2."""
    lam, loc, (best, at) = oracle.lebesgue_max(inputs.equispaced(3), 2, samples=63, rounds=8)
    assert np.all(np.abs(lam - 1.25) <= 4 * U)
    assert np.all(np.abs(np.abs(loc) - 0.5) <= 1e-7)
    assert abs(best - 1.25) <= 4 * U


def _golden_max(fun, a, b, iters=70):
    """Golden-section search for the maximum of a unimodal fun on [a, b]
    (points rounded to binary64, values exact)."""
    phi = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - phi * (b - a), a + phi * (b - a)
    fc, fd = fun(c), fun(d)
    for _ in range(iters):
        if fc >= fd:
            b, d, fd = d, c, fc
            c = b - phi * (b - a)
            fc = fun(c)
        else:
            a, c, fc = c, d, fd
            d = a + phi * (b - a)
            fd = fun(d)
    return (fc, c) if fc >= fd else (fd, d)


@pytest.mark.parametrize("family,n,d", [("equispaced", 7, 0), ("equispaced", 8, 3),
                                        ("cheb2", 7, 2), ("random", 8, 1), ("random", 6, 4)])
def test_fh_against_exact_blend_form(family, n, d):
    nodes = _node_sets(n)[family]
    lam, loc, _ = oracle.lebesgue_max(nodes, d, samples=128, rounds=5)
    for k in range(n - 1):
        fun = lambda t: exact.blend_lebesgue(nodes, d, Fraction(float(t)))  # noqa: E731
        # coarse exact grid first: the golden section needs the right hump
        grid = np.linspace(nodes[k], nodes[k + 1], 41)[1:-1]
        vals = [fun(t) for t in grid]
        i = int(np.argmax([float(v) for v in vals]))
        a = grid[i - 1] if i > 0 else nodes[k]
        b = grid[i + 1] if i < grid.size - 1 else nodes[k + 1]
        v, t = _golden_max(fun, a, b)
        v = float(v)
        assert abs(lam[k] - v) <= _tol(v), (family, k, lam[k], v)
        assert abs(loc[k] - t) <= 1e-5 * (nodes[k + 1] - nodes[k]), (family, k, loc[k], t)


@pytest.mark.parametrize("d", [0, 1])
def test_two_nodes_is_linear_interpolation(d):
    lam, loc, (best, at) = oracle.lebesgue_max(np.array([-0.75, 2.5]), d, samples=33, rounds=3)
    assert abs(lam[0] - 1.0) <= 4 * U and -0.75 < loc[0] < 2.5


def test_single_node():
    lam, loc, best = oracle.lebesgue_max(np.array([0.25]), 0)
    assert lam.size == 0 and best == (1.0, 0.25)


@pytest.mark.parametrize("e", [-30, 7, 200])
def test_power_of_two_scaling_is_exact(e):
    nodes = inputs.jittered_nodes(65, np.random.default_rng(5), rel=0.2)
    lam, loc, _ = oracle.lebesgue_max(nodes, 4, samples=96, rounds=4)
    lam2, loc2, _ = oracle.lebesgue_max(np.ldexp(nodes, e), 4, samples=96, rounds=4)
    assert np.array_equal(lam, lam2)
    assert np.array_equal(np.ldexp(loc, e), loc2)


def test_symmetric_nodes_give_mirrored_maxima():
    for nodes, d in ((inputs.equispaced(101), 3), (inputs.cheb2(40), 2)):
        lam, loc, _ = oracle.lebesgue_max(nodes, d)
        assert np.all(np.abs(lam - lam[::-1]) <= 1e-13 * lam)
        assert np.all(np.abs(loc + loc[::-1]) <= 1e-6 * np.diff(nodes))


def test_more_rounds_never_lower_a_maximum():
    nodes = inputs.cheb2(60)
    prev = None
    for r in range(1, 7):
        lam, _, _ = oracle.lebesgue_max(nodes, 3, samples=16, rounds=r)
        if prev is not None:
            assert np.all(lam >= prev)
        prev = lam


def test_dense_random_sample_never_exceeds_the_maximum():
    g = np.random.default_rng(9)
    for nodes, d in ((inputs.equispaced(41), 3), (inputs.cheb2(33), 2),
                     (inputs.jittered_nodes(50, g, rel=0.3), 5)):
        lam, _, (best, _) = oracle.lebesgue_max(nodes, d)
        pts = g.uniform(nodes[0], nodes[-1], 200000)
        _, lam_p, _ = oracle.evaluate(nodes, np.zeros_like(nodes), d, pts)
        k = np.clip(np.searchsorted(nodes, pts) - 1, 0, nodes.size - 2)
        assert np.all(lam_p <= lam[k] * (1 + 1e-13))
        # and the dense sample comes close to it (the maxima are smooth humps)
        assert lam_p.max() >= best * (1 - 1e-6)


def test_errors():
    nodes = inputs.equispaced(5)
    for kw in ({"samples": 0}, {"rounds": 0}):
        with pytest.raises(oracle.OracleError):
            oracle.lebesgue_max(nodes, 2, **kw)
    with pytest.raises(oracle.OracleError):
        oracle.lebesgue_max(nodes, 5)


def test_interval_subset_gives_the_same_values():
    nodes = inputs.jittered_nodes(300, np.random.default_rng(3), rel=0.3)
    lam, loc, _ = oracle.lebesgue_max(nodes, 4, samples=64, rounds=3)
    ks = np.array([298, 0, 17, 150, 17])
    lam2, loc2, (best, at) = oracle.lebesgue_max(nodes, 4, samples=64, rounds=3, intervals=ks)
    assert np.array_equal(lam2, lam[ks]) and np.array_equal(loc2, loc[ks])
    assert best == lam[ks].max()
    with pytest.raises(oracle.OracleError):
        oracle.lebesgue_max(nodes, 4, intervals=[299])
