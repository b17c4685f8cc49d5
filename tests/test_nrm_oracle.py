"""Pins of the normalization oracle (oracle/nrm_oracle.c) to facts that do
not come from the oracle itself:

- the Table 2 parameters satisfy conditions condA-condF exactly (exact
  rational arithmetic on the IEEE format constants), and the closed form
  (tau) of Section 2 is checked against them;
- Lemma 1 (vectors in R^2 and R^3) and Lemma 2 (quaternions): the bounds on
  the direction, the angle, the length and the products q_i q_j, against
  80-digit decimal references, over inputs spanning the whole exponent
  range of binary32 and binary64;
- the 2.5 u bound on the sum-of-squares length when the largest entry lies
  in [tau_min, tau_max], and bit-for-bit agreement with the naive formula
  there (the scale factor is then 1);
- invariance under power-of-two scaling of the input (exact scaling, fact
  (rndA) of the proofs appendix);
- zero vectors, NaN propagation, finiteness for finite input;
- the quotient algorithms and the naive formula on cases with known
  answers.
"""
import decimal
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import nrm
from paper_1606_06508_amd import inputs

D = decimal.Decimal
CTX = decimal.Context(prec=80, Emax=10 ** 6, Emin=-10 ** 6)

# IEEE binary32 / binary64: unit roundoff u, smallest subnormal alpha,
# smallest normal nu, largest finite omega (exact rationals).
FMT = {
    np.float32: dict(u=Fraction(1, 2 ** 24), alpha=Fraction(1, 2 ** 149), nu=Fraction(1, 2 ** 126),
                     omega=(2 - Fraction(1, 2 ** 23)) * 2 ** 127),
    np.float64: dict(u=Fraction(1, 2 ** 53), alpha=Fraction(1, 2 ** 1074),
                     nu=Fraction(1, 2 ** 1022), omega=(2 - Fraction(1, 2 ** 52)) * 2 ** 1023),
}
TABLE2 = {np.float32: (2.0 ** -49, 2.0 ** 100, 2.0 ** 62, 2.0 ** -66),
          np.float64: (2.0 ** -482, 2.0 ** 592, 2.0 ** 510, 2.0 ** -514)}
DTYPES = (np.float32, np.float64)


@pytest.fixture(autouse=True)
def _decimal_context():
    """Every decimal operation of these tests runs at 80 digits."""
    with decimal.localcontext(CTX):
        yield


def _dec(v):
    return CTX.create_decimal(float(v))


def _exact(x):
    """(r, x / r) of one vector as 80-digit decimals."""
    xs = [_dec(v) for v in x]
    r = CTX.sqrt(sum((CTX.multiply(v, v) for v in xs), D(0)))
    return r, [CTX.divide(v, r) for v in xs]


# ---------------------------------------------------------- parameters --
@pytest.mark.parametrize("dt", DTYPES)
def test_table2_parameters_are_the_oracles(dt):
    assert nrm.params(dt) == TABLE2[dt]


@pytest.mark.parametrize("dt", DTYPES)
def test_table2_satisfies_conditions(dt):
    f = FMT[dt]
    u, alpha, nu, omega = f["u"], f["alpha"], f["nu"], f["omega"]
    tmin, smin, tmax, smax = (Fraction(v) for v in TABLE2[dt])
    # condA: fl(nu^2) = 0, u^2 >= 16 alpha, u <= 1e-6
    nu_f = dt(float(nu))
    assert dt(nu_f * nu_f) == 0
    assert u * u >= 16 * alpha and u <= Fraction(1, 10 ** 6)
    # condB: sigma_min and sigma_max are powers of two
    for s in (smin, smax):
        assert math.frexp(float(s))[0] == 0.5
    # condC, condD
    assert u * u * tmin * tmin >= alpha and 8 * tmax * tmax <= omega
    assert omega * tmin >= 1 and 3 * nu * tmax <= 1
    # condE: sigma_min x in [tau_min, tau_max] for every float x in (0, tau_min]
    # (the product is exact and monotone: check the ends)
    assert smin * alpha >= tmin and smin * tmin <= tmax
    # condF: sigma_max x in [tau_min, tau_max] for x in [tau_max, omega]
    assert smax * tmax >= tmin and smax * omega <= tmax


@pytest.mark.parametrize("dt", DTYPES)
def test_closed_form_tau(dt):
    """The closed form (tau) of Section 2 gives Table 2's tau_max, and a
    tau_min one binade (binary32) or two binades (binary64) below Table 2's,
    which also satisfies condC; the oracle takes Table 2's values."""
    f = FMT[dt]
    tmin_cf = 2.0 ** math.ceil(math.log2(f["alpha"] / f["u"] ** 2) / 2)
    tmax_cf = 2.0 ** math.floor((math.log2(f["omega"]) - 3) / 2)
    assert tmax_cf == TABLE2[dt][2]
    assert tmin_cf == (2.0 ** -50 if dt == np.float32 else 2.0 ** -484)
    assert f["u"] ** 2 * Fraction(tmin_cf) ** 2 >= f["alpha"]


# -------------------------------------------------------------- lemmas --
def _lemma_cases(dim, dt, n=600):
    x = inputs.nrm_vectors(n, dim, dt, salt=7, zero_frac=0.0, nan_frac=0.0)
    # add vectors at the extremes: all components tiny subnormals, all
    # near the largest finite value, a single nonzero entry
    lo, hi, _ = inputs._format(dt)
    extra = np.array([[2.0 ** lo] * dim, [-(2.0 ** lo)] + [2.0 ** (lo + 1)] * (dim - 1),
                      [2.0 ** hi * 1.5] * dim, [0.0] * (dim - 1) + [2.0 ** (lo + 3)],
                      [2.0 ** hi] + [0.0] * (dim - 1)], dtype=np.float64).astype(dt)
    return np.concatenate([x, extra])


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dim", [2, 3])
def test_lemma1_vectors(dim, dt):
    f = FMT[dt]
    u, alpha, nu, omega = (_dec(f[k]) if k != "omega" else CTX.create_decimal(float(f[k]))
                           for k in ("u", "alpha", "nu", "omega"))
    x = _lemma_cases(dim, dt)
    r_hat, x_hat = nrm.normalize(x, "scaling")
    for i in range(x.shape[0]):
        r, xbar = _exact(x[i])
        assert np.all(np.isfinite(x_hat[i])) and r_hat[i] != 0
        xh = [_dec(v) for v in x_hat[i]]
        err = CTX.sqrt(sum(((a - b) ** 2 for a, b in zip(xh, xbar)), D(0)))
        assert err <= (D("3.001") + D(dim) / 2) * u, (i, x[i])
        # angle between x and x_hat: sin^2 = 1 - cos^2
        dot = sum((a * b for a, b in zip(xh, xbar)), D(0))
        nh = CTX.sqrt(sum((a * a for a in xh), D(0)))
        cos = dot / nh
        sin = CTX.sqrt(max(D(0), 1 - cos * cos))
        assert sin <= D("1.001") * u, (i, x[i])
        if (1 + (1 + D(dim) / 2) * u) * r <= omega:
            assert np.isfinite(r_hat[i])
            bound = (1 + D(dim) / 2) * r * u + (alpha / 2 if 2 * r <= 3 * nu / 2 else 0)
            assert abs(_dec(r_hat[i]) - r) <= bound, (i, x[i])


@pytest.mark.parametrize("dt", DTYPES)
def test_lemma2_quaternions(dt):
    f = FMT[dt]
    u, alpha, nu, omega = (CTX.create_decimal(float(f[k])) for k in ("u", "alpha", "nu", "omega"))
    q = np.concatenate([_lemma_cases(4, dt), inputs.near_unit_quaternions(200, dt, salt=3)])
    r_hat, q_hat = nrm.normalize(q, "scaling")
    for i in range(q.shape[0]):
        r, qbar = _exact(q[i])
        assert np.all(np.isfinite(q_hat[i])) and r_hat[i] != 0
        qh = [_dec(v) for v in q_hat[i]]
        err = CTX.sqrt(sum(((a - b) ** 2 for a, b in zip(qh, qbar)), D(0)))
        assert err <= D("5.001") * u, (i, q[i])
        if (1 + 3 * u) * r <= omega:
            assert np.isfinite(r_hat[i])
            bound = 3 * r * u + (alpha / 2 if 2 * r <= 3 * nu / 2 else 0)
            assert abs(_dec(r_hat[i]) - r) <= bound, (i, q[i])
        for a in range(4):
            for b in range(4):
                lhs = abs(qh[a] * qh[b] - qbar[a] * qbar[b])
                assert lhs <= (D("1.001") + D("8.001") * abs(qbar[a] * qbar[b])) * u, (i, a, b)


# ------------------------------------------------------- in-range facts --
def _in_range(dt, dim, n=2000, salt=11):
    """Vectors whose largest entry lies in [tau_min, tau_max]."""
    g = np.random.default_rng(salt)
    tmin, _, tmax, _ = TABLE2[dt]
    e = g.integers(int(math.log2(tmin)), int(math.log2(tmax)), size=(n, 1))
    x = np.ldexp(g.uniform(-2, 2, size=(n, dim)), e - g.integers(0, 30, size=(n, dim)))
    x = x.astype(dt)
    m = np.abs(x).max(axis=1)
    return x[(m >= tmin) & (m <= tmax)]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dim", [2, 3, 4])
def test_in_range_length_bound_and_naive_agreement(dim, dt):
    u = CTX.create_decimal(float(FMT[dt]["u"]))
    x = _in_range(dt, dim)
    r_s, xh_s = nrm.normalize(x, "scaling")
    r_n, xh_n = nrm.normalize(x, "naive")
    assert np.array_equal(r_s.view(np.uint8), r_n.view(np.uint8))
    assert np.array_equal(xh_s.view(np.uint8), xh_n.view(np.uint8))
    for i in range(0, x.shape[0], 7):
        r, _ = _exact(x[i])
        assert abs(_dec(r_n[i]) - r) <= D("2.5") * u * r


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dim", [2, 3, 4])
def test_power_of_two_scaling_invariance(dim, dt):
    """x -> 2^k x (exact while every entry stays normal) leaves x_hat bit
    for bit unchanged and multiplies r_hat by 2^k exactly."""
    g = np.random.default_rng(5 + dim)
    lo, hi, _ = inputs._format(dt)
    nu = 2.0 ** (-126 if dt == np.float32 else -1022)
    base = np.ldexp(g.uniform(1, 2, size=(400, dim)) * g.choice([-1, 1], size=(400, dim)),
                    g.integers(-20, 20, size=(400, dim))).astype(dt)
    r0, xh0 = nrm.normalize(base, "scaling")
    checked = 0
    for k in (-(hi - 30), -100, -7, 13, 100, hi - 30):
        xs = np.ldexp(base.astype(np.float64), k).astype(dt)
        ok = np.all((np.abs(xs) >= nu) & np.isfinite(xs), axis=1)
        r1, xh1 = nrm.normalize(xs[ok], "scaling")
        assert np.array_equal(xh1, xh0[ok]), k
        assert np.array_equal(r1, np.ldexp(r0[ok].astype(np.float64), k).astype(dt)), k
        checked += int(ok.sum())
    assert checked > 1000


# ------------------------------------------------------- special inputs --
@pytest.mark.parametrize("dt", DTYPES)
def test_zero_nan_inf(dt):
    for dim in (2, 3, 4):
        z = np.zeros((1, dim), dtype=dt)
        r, xh = nrm.normalize(z, "scaling")
        want = [0.0] * dim
        if dim == 4:
            want[2] = 1.0  # the zero quaternion's direction
        assert r[0] == 0 and np.array_equal(xh[0], np.array(want, dtype=dt))
        for k in range(dim):
            for other in (0.0, 1.0, 1e-30, 3e30):
                v = np.full((1, dim), other, dtype=dt)
                v[0, k] = np.nan
                r, xh = nrm.normalize(v, "scaling")
                assert np.isnan(r[0]) and np.all(np.isnan(xh[0])), (dim, k, other)
        # finite input, finite output (also next to the overflow threshold)
        big = np.full((1, dim), np.finfo(dt).max, dtype=dt)
        r, xh = nrm.normalize(big, "scaling")
        assert np.all(np.isfinite(xh)) and np.isinf(r[0])  # ||x|| itself overflows
        np.testing.assert_allclose(xh[0].astype(np.float64), 1 / math.sqrt(dim), rtol=4e-7)


@pytest.mark.parametrize("dt", DTYPES)
def test_other_methods_known_answers(dt):
    x = np.array([[3.0, 4.0], [-6.0, 8.0]], dtype=dt)
    for method in ("scaling", "quotient", "naive"):
        r, xh = nrm.normalize(x, method)
        rtol = 0 if method in ("scaling", "naive") else 3 * float(FMT[dt]["u"])
        np.testing.assert_allclose(r, [5.0, 10.0], rtol=rtol, atol=0, err_msg=method)
        # h = 1/r, then h x: two roundings, within 2u of x/r
        np.testing.assert_allclose(xh, [[0.6, 0.8], [-0.6, 0.8]], rtol=2 * float(FMT[dt]["u"]),
                                   err_msg=method)
    x3 = np.array([[2.0, 3.0, 6.0], [-6.0, 2.0, 3.0], [0.0, 0.0, 0.0], [1.0, 4.0, 8.0]],
                  dtype=dt)
    for method in ("scaling", "quotient", "quotient_pivot", "naive"):
        r, xh = nrm.normalize(x3, method)
        # exact squares and square roots: scaling and naive are exact; the
        # quotient algorithms round x/m first (an ulp or two)
        rtol = 0 if method in ("scaling", "naive") else 3 * float(FMT[dt]["u"])
        np.testing.assert_allclose(r[[0, 1, 3]], np.array([7.0, 7.0, 9.0]), rtol=rtol, atol=0,
                                   err_msg=method)
        np.testing.assert_allclose(xh[0], np.array([2, 3, 6]) / 7, rtol=4 * float(FMT[dt]["u"]))
        np.testing.assert_allclose(xh[3], np.array([1, 4, 8]) / 9, rtol=4 * float(FMT[dt]["u"]))
        if method != "naive":
            assert r[2] == 0 and np.array_equal(xh[2], np.zeros(3, dtype=dt)), method
    # the naive formula overflows / underflows where scaling does not
    tiny = np.array([[1e-200, 1e-200]], dtype=np.float64)
    r_n, xh_n = nrm.normalize(tiny, "naive")
    r_s, xh_s = nrm.normalize(tiny, "scaling")
    assert r_n[0] == 0 and np.all(~np.isfinite(xh_n))
    np.testing.assert_allclose(r_s[0], math.sqrt(2) * 1e-200, rtol=1e-15)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("method", ["quotient", "quotient_pivot"])
def test_quotient_algorithms_accuracy(method, dt):
    """The quotient algorithms reach the same length and direction within a
    few units of roundoff over the whole exponent range."""
    u = float(FMT[dt]["u"])
    x = inputs.nrm_vectors(3000, 3, dt, salt=13, zero_frac=0.0, nan_frac=0.0)
    r_q, xh_q = nrm.normalize(x, method)
    r_s, xh_s = nrm.normalize(x, "scaling")
    fin = np.isfinite(r_q) & np.isfinite(r_s)
    # subnormal lengths carry an absolute quantum alpha (the alpha/2 of the lemmas)
    np.testing.assert_allclose(r_q[fin].astype(np.float64), r_s[fin].astype(np.float64),
                               rtol=8 * u, atol=2 * float(FMT[dt]["alpha"]))
    assert np.max(np.abs(xh_q.astype(np.float64) - xh_s.astype(np.float64))) <= 10 * u


def test_argument_errors():
    with pytest.raises(nrm.OracleError):
        nrm.normalize(np.zeros((2, 2)), "quotient_pivot")  # Algorithm 2 is three dimensional
    with pytest.raises(ValueError):
        nrm.normalize(np.zeros((2, 2), dtype=np.int32))
