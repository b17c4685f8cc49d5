"""Parity of the HIP evaluation path (weights, fused second-form sum with the
exact-hit branch, Lebesgue function) against the FP64 oracle, through the C
ABI.  Sizes span several node groups and point blocks with ragged tails;
full-size workloads are checked on sampled outputs."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _np(t):
    return t.cpu().numpy()


def _run(nodes, values, d, pts, precision="fp64", lebesgue=True, weights=None):
    out = fh.evaluate(_t(nodes), _t(values), d, _t(pts), lebesgue=lebesgue,
                      precision=precision, weights=None if weights is None else _t(weights))
    torch.cuda.synchronize()
    if lebesgue:
        return _np(out[0]), _np(out[1])
    return _np(out), None


def _check_case(nodes, values, d, pts, precision="fp64", tol=metrics.FP64_TOL, lam_metric="rel"):
    r, lam = _run(nodes, values, d, pts, precision)
    r_o, lam_o, s_o = oracle.evaluate(nodes, values, d, pts)
    stats = metrics.parity(r, lam, r_o, lam_o, s_o)
    metrics.check_fp64(stats, tol, lam_metric)
    # exact hits: bit-for-bit values and Lambda == 1
    hit = np.isin(pts, nodes)
    if np.any(hit):
        idx = np.searchsorted(nodes, pts[hit])
        assert np.array_equal(r[hit].view(np.int64), np.asarray(values)[idx].view(np.int64))
        assert np.all(lam[hit] == 1.0)
    return stats


# ------------------------------------------------------------- weights --
@pytest.mark.parametrize("family,n,d", [("equi", 21, 3), ("equi", 1001, 0), ("equi", 1001, 8),
                                        ("cheb", 777, 5), ("jitter", 4097, 6), ("equi", 1, 0),
                                        ("cheb", 11, 10), ("equi", 2049, 4)])
def test_weights_bitwise(family, n, d):
    g = np.random.default_rng(n + d)
    x = {"equi": inputs.equispaced, "cheb": inputs.cheb2}.get(family, None)
    nodes = x(n) if x else inputs.jittered_nodes(n, g)
    w = _np(fh.weights(_t(nodes), d))
    w_o = oracle.weights(nodes, d)
    assert np.array_equal(w.view(np.int64), w_o.view(np.int64))


# ---------------------------------------------------------- workloads --
def test_runge_full():
    """The Runge workload in full: besides the bars, plain relative error
    e_rel(r) <= 1e-13 at every point, without the conditioning filter (its
    r = 1/(1+25x^2) stays away from zero)."""
    c = inputs.runge()
    st = _check_case(c["nodes"], c["values"], c["d"], c["points"])
    assert st["e_rel_max"] <= metrics.FP64_TOL, st
    assert st["n_beyond_lam_max"] == 0 and st["nan_mismatch_r"] == 0, st


@pytest.mark.parametrize("d", list(range(9)))
def test_sines_reduced(d):
    c = inputs.sines_workload(m=20011)
    _check_case(c["nodes"], c["values"], d, c["points"])


def test_split_workload_fp64_reduced():
    c = inputs.split_workload(m=30011)
    _check_case(c["nodes"], c["values"], c["d"], c["points"])


def test_grad_workload_forward_reduced():
    c = inputs.grad_workload(m=25013)
    _check_case(c["nodes"], c["values"], c["d"], c["points"])


@pytest.mark.parametrize("d", [0, 4, 8])
def test_sines_full_size_sampled(d):
    """Full 10^6 points in the benchmark's launch configuration; the oracle
    checks a seeded sample of 3000 outputs one by one."""
    c = inputs.sines_workload()
    r, lam = _run(c["nodes"], c["values"], d, c["points"])
    idx = np.random.default_rng(d).choice(c["points"].size, 3000, replace=False)
    r_o, lam_o, s_o = oracle.evaluate(c["nodes"], c["values"], d, c["points"][idx])
    metrics.check_fp64(metrics.parity(r[idx], lam[idx], r_o, lam_o, s_o))


def test_split_workload_full_size_fp64_sampled():
    c = inputs.split_workload()
    r, lam = _run(c["nodes"], c["values"], c["d"], c["points"])
    idx = np.random.default_rng(3).choice(c["points"].size, 2000, replace=False)
    r_o, lam_o, s_o = oracle.evaluate(c["nodes"], c["values"], c["d"], c["points"][idx])
    metrics.check_fp64(metrics.parity(r[idx], lam[idx], r_o, lam_o, s_o))


# -------------------------------------------------------------- shapes --
@pytest.mark.parametrize("m", [1, 2, 63, 64, 65, 255, 257, 1023, 1025, 4097, 262145])
def test_ragged_point_counts(m):
    g = np.random.default_rng(m)
    nodes = inputs.cheb2(70)
    vals = g.standard_normal(70)
    pts = g.uniform(-1, 1, size=m)
    _check_case(nodes, vals, 3, pts, lam_metric="cond")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 64, 65, 127, 129])
def test_node_counts(n):
    g = np.random.default_rng(1000 + n)
    nodes = inputs.equispaced(n)
    vals = g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1.2, 1.2, size=3001), nodes])
    # d = n-1 on many equispaced nodes is polynomial interpolation with a
    # Lebesgue constant near 2^n: beyond the oracle's own precision (its
    # compensated D is good to about u|D| + n u^2 L), so the degree is capped
    for d in sorted({0, min(2, n - 1), min(n - 1, 12)}):
        _check_case(nodes, vals, d, pts, lam_metric="cond")


def test_empty_point_set():
    c = inputs.runge()
    r = fh.evaluate(_t(c["nodes"]), _t(c["values"]), 3, torch.empty(0, dtype=torch.float64,
                                                                     device=DEV))
    torch.cuda.synchronize()
    assert r.numel() == 0


def test_special_points():
    c = inputs.runge()
    nodes, vals = c["nodes"], c["values"]
    pts = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, nodes[0], nodes[-1], 1e300, -1e300, 1e-300,
                    np.nextafter(nodes[5], 2.0), 5.0, -7.5, 1e-200, 2.0 ** -1000])
    r, lam = _run(nodes, vals, 3, pts)
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, 3, pts)
    assert np.array_equal(np.isnan(r), np.isnan(r_o))
    assert np.array_equal(np.isnan(lam), np.isnan(lam_o))
    fin = ~np.isnan(r_o)
    assert np.all(np.abs(r[fin] - r_o[fin]) <= 1e-13 * s_o[fin])
    # far outside the nodes D cancels heavily (Lambda ~ 1e6 .. 1e17 here), so
    # Lambda is held to the conditioned bar
    assert np.all(np.abs(lam[fin] - lam_o[fin]) <= 1e-13 * lam_o[fin] * (1 + lam_o[fin]))
    assert r[3] == vals[10] and r[4] == vals[10] and lam[3] == 1.0


def test_nan_value_poisons_all_but_other_hits():
    c = inputs.runge()
    f = c["values"].copy()
    f[4] = np.nan
    pts = np.concatenate([[0.123, -0.77], c["nodes"]])
    r, _ = _run(c["nodes"], f, 3, pts)
    assert np.isnan(r[0]) and np.isnan(r[1]) and np.isnan(r[2 + 4])
    others = np.delete(np.arange(21), 4)
    assert np.array_equal(r[2 + others], f[others])


def test_lebesgue_only_matches_fused():
    c = inputs.sines_workload(n=301, m=9001)
    xn, t = _t(c["nodes"]), _t(c["points"])
    lam1 = _np(fh.lebesgue(xn, 5, t))
    _, lam2 = _run(c["nodes"], c["values"], 5, c["points"])
    _, lam_o, _ = oracle.evaluate(c["nodes"], c["values"], 5, c["points"])
    assert np.array_equal(lam1, lam2)
    assert np.max(np.abs(lam1 - lam_o) / lam_o) <= 1e-13


def test_value_only_matches_fused():
    c = inputs.sines_workload(n=301, m=9001)
    r1, _ = _run(c["nodes"], c["values"], 5, c["points"], lebesgue=False)
    r2, _ = _run(c["nodes"], c["values"], 5, c["points"], lebesgue=True)
    assert np.array_equal(r1, r2)


def test_given_weights_and_power_of_two_scaling():
    """Passing fh_weights' output reproduces the internal pass bit-for-bit, and
    scaling all weights by 2^e leaves r and Lambda unchanged bit-for-bit
    (every product w t scales exactly)."""
    c = inputs.sines_workload(n=501, m=7001)
    w = oracle.weights(c["nodes"], 4)
    r0, l0 = _run(c["nodes"], c["values"], 4, c["points"])
    r1, l1 = _run(c["nodes"], c["values"], 4, c["points"], weights=w)
    r2, l2 = _run(c["nodes"], c["values"], 4, c["points"], weights=np.ldexp(w, -77))
    assert np.array_equal(r0, r1) and np.array_equal(l0, l1)
    assert np.array_equal(r0, r2) and np.array_equal(l0, l2)


def test_deterministic():
    c = inputs.split_workload(m=50000)
    a = _run(c["nodes"], c["values"], 6, c["points"])
    b = _run(c["nodes"], c["values"], 6, c["points"])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------ device checks --
@pytest.mark.parametrize("nodes,code", [([0.0, 0.5, 0.5, 1.0], fh.FH_E_NODES),
                                        ([0.0, 1.0, 0.5], fh.FH_E_NODES),
                                        ([0.0, np.nan, 1.0], fh.FH_E_NONFINITE),
                                        ([0.0, 0.5, np.inf], fh.FH_E_NONFINITE)])
def test_device_node_checks(nodes, code):
    ws = fh.Workspace(DEV)
    x = _t(np.array(nodes))
    fh.evaluate(x, _t(np.zeros(len(nodes))), 1, _t(np.array([0.25])), ws=ws)
    st, bits = ws.status()
    assert st == code and bits != 0
    st, bits = ws.status()          # sticky bits are cleared by the read
    assert st == fh.FH_OK and bits == 0


def test_bad_arguments_raise():
    c = inputs.runge()
    with pytest.raises(fh.FhError) as e:
        fh.evaluate(_t(c["nodes"]), _t(c["values"]), 21, _t(c["points"]))
    assert e.value.code == fh.FH_E_DEGREE
    with pytest.raises(TypeError):
        fh.evaluate(_t(c["nodes"]).float(), _t(c["values"]), 3, _t(c["points"]))


# ------------------------------------------------------------ variants --
@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_every_kernel_variant(precision):
    """Every launch variant the tuner may pick meets the same bar (binary64
    bar for fp64; the split form's stated bound for split)."""
    g = np.random.default_rng(11)
    nodes = inputs.jittered_nodes(333, g)
    vals = g.standard_normal(333)
    pts = np.concatenate([g.uniform(-1, 1, size=5003), nodes[::7], nodes[5::50] + 1e-9])
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, 5, pts)
    try:
        for vid, p, grp, s in fh.variants(precision):
            fh.tune_force(precision, vid)
            r, lam = _run(nodes, vals, 5, pts, precision)
            if precision == "fp64":
                metrics.check_fp64(metrics.parity(r, lam, r_o, lam_o, s_o))
            else:
                metrics.check_split(metrics.parity(r, lam, r_o, lam_o, s_o,
                                                   metrics.SPLIT_LAMBDA_MAX))
            hit = np.isin(pts, nodes)
            assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
            assert np.all(lam[hit] == 1.0), vid
    finally:
        fh.tune_force(precision, -1)
