"""The derivative output (fh_eval_deriv): r' against the oracle's r'
(e_cond(r') = |r'_HIP - r'_oracle| / S', S' the oracle's error scale of r'),
binary64 and FP32-split, at points whose Lebesgue function is within the
cutoffs of the parity bars; exact hits (node formula); non-finite points;
bit-identity with the adjoint's dL/dx_p for g = 1 (the same per-point pass);
polynomial reproduction."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"fp64": 1e-12, "split": metrics.SPLIT_TOL}
# the split derivative kernel has no conditioning guard: the binary32 band
LAM_MAX = {"fp64": metrics.FP64_LAMBDA_MAX, "split": metrics.SPLIT_TERMS_LAMBDA_MAX}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _deriv(nodes, vals, d, pts, precision="fp64", weights=None):
    r, dr = fh.eval_deriv(_t(nodes), _t(vals), d, _t(pts), precision=precision,
                          weights=None if weights is None else _t(weights))
    torch.cuda.synchronize()
    return r.cpu().numpy(), dr.cpu().numpy()


def _check(nodes, vals, d, pts, precision):
    r, dr = _deriv(nodes, vals, d, pts, precision)
    r_o, dr_o, s_o = oracle.eval_deriv(nodes, vals, d, pts)
    _, lam_o, _ = oracle.evaluate(nodes, vals, d, pts)
    fin = np.isfinite(pts)
    assert np.all(np.isnan(dr[~fin])) and np.all(np.isnan(r[~fin]))
    keep = fin & ~(lam_o > LAM_MAX[precision])
    diff = np.abs(dr[keep] - dr_o[keep])
    # an empty node-formula sum (one node) has r' = 0 and scale 0
    with np.errstate(invalid="ignore", divide="ignore"):
        err = np.where(s_o[keep] > 0, diff / s_o[keep], np.where(diff == 0, 0.0, np.inf))
    assert err.max() <= TOL[precision], (precision, err.max())
    hit = np.isin(pts, nodes)
    assert np.array_equal(r[hit], r_o[hit])
    return err.max()


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("d", [0, 3, 8])
def test_sines_reduced(d, precision):
    c = inputs.sines_workload(m=20011)
    pts = np.concatenate([c["points"], c["nodes"][::37], [np.nan, np.inf, -np.inf]])
    e = _check(c["nodes"], c["values"], d, pts, precision)
    if precision == "split":
        assert e > 1e-13  # the binary32 path ran


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("n,d", [(1, 0), (2, 1), (5, 4), (64, 3), (129, 10)])
def test_shapes(n, d, precision):
    g = np.random.default_rng(500 + n + d)
    nodes = inputs.equispaced(n) if n > 1 else np.array([0.3])
    vals = g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1.05, 1.05, 2000), nodes, nodes[-1:] + 1e-13])
    _check(nodes, vals, d, pts, precision)


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_matches_adjoint_point_gradient_bitwise(precision):
    """r' is the adjoint's dL/dx_p for g = 1, computed by the same per-point
    pass: the same bits."""
    c = inputs.grad_workload(n=513, m=30011)
    _, dr = _deriv(c["nodes"], c["values"], c["d"], c["points"], precision)
    _, gx, _ = fh.eval_backward(_t(c["nodes"]), _t(c["values"]), c["d"], _t(c["points"]),
                                torch.ones(c["points"].size, dtype=torch.float64, device=DEV),
                                need_values=False, need_nodes=False, precision=precision)
    torch.cuda.synchronize()
    assert np.array_equal(dr, gx.cpu().numpy())


def test_polynomial_reproduction_and_given_weights():
    g = np.random.default_rng(12)
    nodes = inputs.equispaced(301)
    for d in (1, 4, 7):
        coef = g.standard_normal(d + 1)
        vals = np.polyval(coef, nodes)
        pts = g.uniform(-1, 1, 5000)
        _, dr = _deriv(nodes, vals, d, pts)
        want = np.polyval(np.polyder(coef), pts)
        _, _, s_o = oracle.eval_deriv(nodes, vals, d, pts)
        assert np.all(np.abs(dr - want) <= 1e-12 * s_o)
        w = oracle.weights(nodes, d)
        _, dr2 = _deriv(nodes, vals, d, pts, weights=np.ldexp(w, -40))
        assert np.array_equal(dr, dr2)  # a power-of-two weight scale cancels exactly


def test_value_only_output_may_be_omitted():
    c = inputs.sines_workload(m=1000)
    r1, dr1 = fh.eval_deriv(_t(c["nodes"]), _t(c["values"]), 4, _t(c["points"]))
    r2, dr2 = fh.eval_deriv(_t(c["nodes"]), _t(c["values"]), 4, _t(c["points"]), want_r=False)
    torch.cuda.synchronize()
    assert r2 is None and torch.equal(dr1, dr2)
