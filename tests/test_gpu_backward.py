"""Parity of the HIP adjoint (fh_eval_backward) with the FP64 oracle, the
structural identities of the gradients at full size, central differences
of the HIP forward pass, and the autograd front.

Error scales.  Each gradient component is a sum of terms; its rounding error
is bounded by a few u times the sum of the terms' absolute values (and by
the number of terms in the worst case).  Every term carries c_p = g_p / D_p,
and D_p = sum_k a_pk has condition number Lambda(x_p), so c_p itself is only
known to about u (1 + Lambda(x_p)); each point's terms are weighted by that
factor.  The tests compute those absolute sums independently with numpy and
require |HIP - oracle| <= TOL * scale, TOL = 1e-12 (about 10^4 u: room for
the plain, chunked sums of the kernel over up to 10^4 terms against the
oracle's compensated ones); the scales are metrics.grad_scales.
"""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs
from paper_1606_06508_amd.autograd import FhEval, interpolate

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U = 2.0 ** -53
TOL = metrics.GRAD_TOL


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _np(t):
    return None if t is None else t.cpu().numpy()


def _gpu_bwd(nodes, vals, d, pts, g, saved=False):
    """The two-pass adjoint (fh_eval_backward, saved falsy), or the
    saved-state one (fh_eval_forward, then fh_eval_backward_saved): saved
    "fused" without the derivative (dL/dx_p from the fused pass), "deriv"
    with it (dL/dx_p = g_p r'(x_p) from the forward)."""
    if saved:
        _, st = fh.eval_forward(_t(nodes), _t(vals), d, _t(pts), derivative=saved == "deriv")
        gv, gx, gn = fh.eval_backward_saved(st, _t(g))
    else:
        gv, gx, gn = fh.eval_backward(_t(nodes), _t(vals), d, _t(pts), _t(g))
    torch.cuda.synchronize()
    return _np(gv), _np(gx), _np(gn)


MODES = pytest.mark.parametrize("saved", [False, "fused", "deriv"],
                                ids=["two_pass", "saved", "saved_deriv"])


def _check_against_oracle(nodes, vals, d, pts, g, dense_chain=True, saved=False):
    gv, gx, gn = _gpu_bwd(nodes, vals, d, pts, g, saved)
    o = oracle.backward(nodes, vals, d, pts, g)
    scales = metrics.grad_scales(nodes, vals, d, pts, g)
    err = metrics.grad_errors(gv, gx, gn, o, scales, *((nodes, d) if dense_chain else ()))
    metrics.check_grad(err, TOL)
    return gv, gx, gn, o


# ------------------------------------------------------------- parity --
@MODES
def test_grad_workload_reduced(saved):
    c = inputs.grad_workload(n=513, m=6007)
    _check_against_oracle(c["nodes"], c["values"], c["d"], c["points"], c["grad"], saved=saved)


@MODES
@pytest.mark.parametrize("n,d", [(1, 0), (2, 1), (5, 0), (5, 4), (64, 3), (65, 7), (130, 10)])
def test_shapes_with_hits_and_nan(n, d, saved):
    g = np.random.default_rng(100 + n + d)
    nodes = inputs.equispaced(n) + (g.uniform(-0.2, 0.2, n) * (2.0 / max(n - 1, 1)) if n > 2 else 0)
    nodes = np.sort(nodes)
    vals = g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1.1, 1.1, size=1001), nodes[:: max(1, n // 5)], [np.nan]])
    grad = g.standard_normal(pts.size)
    gv, gx, gn, o = _check_against_oracle(nodes, vals, d, pts, grad, saved=saved)
    assert np.isnan(gx[-1])


@MODES
def test_full_size_identities_and_sampled_points(saved):
    """The full 10^6-point workload: identities that hold at any size, and
    dL/dx_p against the oracle on a seeded sample of points (each dL/dx_p
    depends on its own point only)."""
    c = inputs.grad_workload()
    nodes, vals, d, pts, g = c["nodes"], c["values"], c["d"], c["points"], c["grad"]
    gv, gx, gn = _gpu_bwd(nodes, vals, d, pts, g, saved)
    assert np.all(np.isfinite(gv)) and np.all(np.isfinite(gx)) and np.all(np.isfinite(gn))
    # partition of unity: sum_k dL/df_k = sum_p g_p
    assert abs(gv.sum() - g.sum()) <= 1e-11 * np.abs(g).sum()
    # translation invariance and scale invariance
    tot = gn.sum() + gx.sum()
    assert abs(tot) <= 1e-10 * (np.abs(gn).sum() + np.abs(gx).sum())
    tot = (nodes * gn).sum() + (pts * gx).sum()
    assert abs(tot) <= 1e-10 * (np.abs(nodes * gn).sum() + np.abs(pts * gx).sum())
    idx = np.random.default_rng(5).choice(pts.size, 1500, replace=False)
    o = oracle.backward(nodes, vals, d, pts[idx], g[idx])
    scales = metrics.grad_scales(nodes, vals, d, pts[idx], g[idx])
    metrics.check_grad(metrics.grad_errors(None, gx[idx], None, o, scales), TOL)


@MODES
def test_polynomial_data(saved):
    """Data from a polynomial of degree <= d: dL/dx_p = g_p p'(x_p) and
    dL/dx_k + p'(x_k) dL/df_k = 0."""
    g = np.random.default_rng(3)
    d = 4
    nodes = inputs.equispaced(301)
    poly = g.standard_normal(d + 1)
    vals = np.polyval(poly, nodes)
    pts = g.uniform(-1, 1, size=20000)
    grad = g.standard_normal(pts.size)
    gv, gx, gn = _gpu_bwd(nodes, vals, d, pts, grad, saved)
    dp = grad * np.polyval(np.polyder(poly), pts)
    assert np.allclose(gx, dp, rtol=1e-9, atol=1e-9 * np.abs(dp).max())
    moved = gn + np.polyval(np.polyder(poly), nodes) * gv
    assert np.abs(moved).max() <= 1e-10 * (np.abs(gn).sum() + np.abs(gv).sum())


@MODES
def test_central_differences(saved):
    """Central differences (h = 1e-6) of the HIP forward pass (weights
    recomputed) against the adjoint, within 10 (h^2 M3/6 + 2u sum|g r|/h),
    M3 estimated from differences at 10h."""
    c = inputs.grad_workload(n=257, m=4001)
    nodes, vals, d, pts, g = c["nodes"], c["values"], c["d"], c["points"], c["grad"]
    gv, gx, gn = _gpu_bwd(nodes, vals, d, pts, g, saved)
    xn, f, t, gt = _t(nodes), _t(vals), _t(pts), _t(g)

    def L(nodes_=None, vals_=None, pts_=None):
        r = fh.evaluate(nodes_ if nodes_ is not None else xn, vals_ if vals_ is not None else f,
                        d, pts_ if pts_ is not None else t)
        return float((r * gt).sum())

    r0 = fh.evaluate(xn, f, d, t)
    noise = 2 * U * float((r0 * gt).abs().sum())
    h = 1e-6

    def fd(kind, k, step):
        e = torch.zeros(nodes.size if kind != "pt" else pts.size, dtype=torch.float64, device=DEV)
        e[k] = step
        if kind == "node":
            return (L(nodes_=xn + e) - L(nodes_=xn - e)) / (2 * step)
        if kind == "val":
            return (L(vals_=f + e) - L(vals_=f - e)) / (2 * step)
        return (L(pts_=t + e) - L(pts_=t - e)) / (2 * step)

    for kind, ks, ref in (("node", (0, 1, 77, 128, 255, 256), gn), ("val", (0, 100, 256), gv),
                          ("pt", (0, 17, 4000), gx)):
        for k in ks:
            a, b = fd(kind, k, h), fd(kind, k, 10 * h)
            m3 = abs(b - a) * 6 / (99 * h * h)
            tol = 10 * (h * h * m3 / 6 + noise / h) + 1e-12 * abs(ref[k])
            assert abs(a - ref[k]) <= tol, (kind, k, a, ref[k], tol)


@MODES
def test_deterministic(saved):
    c = inputs.grad_workload(n=1025, m=100003)
    a = _gpu_bwd(c["nodes"], c["values"], c["d"], c["points"], c["grad"], saved)
    b = _gpu_bwd(c["nodes"], c["values"], c["d"], c["points"], c["grad"], saved)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("need", [(True, False, False), (False, True, False), (False, False, True),
                                  (True, True, False), (True, False, True), (False, True, True)])
def test_partial_outputs_match_full(precision, need):
    """Only the requested gradients are computed -- dL/dx_p from the point
    pass alone, dL/df with the first of the four node sums only, the node
    gradient with all of them -- and each has the bits of the full call
    (the same operations in the same order), hits included."""
    c = inputs.grad_workload(n=129, m=5000)
    pts = c["points"].copy()
    pts[:5] = c["nodes"][[0, 3, 64, 100, 128]]                       # exact hits
    args = (_t(c["nodes"]), _t(c["values"]), c["d"], _t(pts), _t(c["grad"]))
    full = fh.eval_backward(*args, precision=precision)
    part = fh.eval_backward(*args, need_values=need[0], need_x=need[1], need_nodes=need[2],
                            precision=precision)
    for want, a, b in zip(need, part, full):
        if want:
            assert torch.equal(a, b)
        else:
            assert a is None


# ------------------------------------------------------------ autograd --
def test_autograd_function_and_gradcheck():
    g = np.random.default_rng(8)
    nodes = _t(np.sort(inputs.equispaced(12) + g.uniform(-0.03, 0.03, 12))).requires_grad_()
    vals = _t(g.standard_normal(12)).requires_grad_()
    x = _t(g.uniform(-1, 1, 25)).requires_grad_()
    assert torch.autograd.gradcheck(lambda a, b, c: FhEval.apply(a, b, c, 3), (nodes, vals, x),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    # backward of a loss equals the adjoint calls: fh_eval_backward without
    # saved state, fh_eval_backward_saved (the default) with it
    w = torch.linspace(-1, 1, 25, dtype=torch.float64, device=DEV)
    r = interpolate(nodes, vals, x, 3, saved=False)
    (r * w).sum().backward()
    gv, gx, gn = fh.eval_backward(nodes.detach(), vals.detach(), 3, x.detach(), w)
    assert torch.equal(nodes.grad, gn) and torch.equal(vals.grad, gv) and torch.equal(x.grad, gx)
    for a in (nodes, vals, x):
        a.grad = None
    r = interpolate(nodes, vals, x, 3)
    (r * w).sum().backward()
    # x requires a gradient: the forward keeps r' (dL/dx = g r')
    r2, st = fh.eval_forward(nodes.detach(), vals.detach(), 3, x.detach(), derivative=True)
    assert torch.equal(r, r2)
    gv, gx, gn = fh.eval_backward_saved(st, w)
    assert torch.equal(nodes.grad, gn) and torch.equal(vals.grad, gv) and torch.equal(x.grad, gx)
    assert torch.autograd.gradcheck(lambda a, b, c: FhEval.apply(a, b, c, 3, "fp64", False),
                                    (nodes, vals, x), eps=1e-6, atol=1e-6, rtol=1e-5)


# ------------------------------------------------- saved-state adjoint --
@pytest.mark.parametrize("derivative", [False, True])
@pytest.mark.parametrize("need", [(True, False, False), (False, True, False), (False, False, True),
                                  (True, True, False), (True, False, True), (False, True, True)])
def test_saved_partial_outputs_match_full(need, derivative):
    """fh_eval_backward_saved computes only what is asked (dL/dx_p alone runs
    the point side of the fused pass without node sums) and each output has
    the bits of the full call, hits and a NaN point included."""
    c = inputs.grad_workload(n=129, m=5000)
    pts = c["points"].copy()
    pts[:5] = c["nodes"][[0, 3, 64, 100, 128]]
    pts[5] = np.nan
    _, st = fh.eval_forward(_t(c["nodes"]), _t(c["values"]), c["d"], _t(pts),
                            derivative=derivative)
    g = _t(c["grad"])
    full = fh.eval_backward_saved(st, g)
    part = fh.eval_backward_saved(st, g, need_values=need[0], need_x=need[1], need_nodes=need[2])
    assert torch.isnan(full[1][5])
    for want, a, b in zip(need, part, full):
        if want:
            assert torch.equal(torch.isnan(a), torch.isnan(b))
            assert torch.equal(a.nan_to_num(0.0), b.nan_to_num(0.0))
        else:
            assert a is None


def test_saved_state_is_reusable():
    """The backward reads the forward's state without changing it: two
    backwards with different loss weights in either order give the same
    bits as each alone."""
    c = inputs.grad_workload(n=300, m=20011)
    _, st = fh.eval_forward(_t(c["nodes"]), _t(c["values"]), c["d"], _t(c["points"]))
    g1 = _t(c["grad"])
    g2 = _t(np.random.default_rng(4).standard_normal(c["points"].size))
    a1 = fh.eval_backward_saved(st, g1)
    a2 = fh.eval_backward_saved(st, g2)
    b1 = fh.eval_backward_saved(st, g1)
    for u, v in zip(a1, b1):
        assert torch.equal(u, v)
    _, st2 = fh.eval_forward(_t(c["nodes"]), _t(c["values"]), c["d"], _t(c["points"]))
    for u, v in zip(a2, fh.eval_backward_saved(st2, g2)):
        assert torch.equal(u, v)


def test_saved_forward_values():
    """r of fh_eval_forward against the oracle at the binary64 bar, hits and
    non-finite points included."""
    c = inputs.grad_workload(n=1025, m=30000)
    pts = c["points"].copy()
    pts[:4] = c["nodes"][[0, 1, 512, 1024]]
    pts[4:7] = [np.nan, np.inf, -np.inf]
    r, _ = fh.eval_forward(_t(c["nodes"]), _t(c["values"]), c["d"], _t(pts))
    r = _np(r)
    ro, lo, so = oracle.evaluate(c["nodes"], c["values"], c["d"], pts[7:])
    assert np.array_equal(r[:4], c["values"][[0, 1, 512, 1024]])
    assert np.all(np.isnan(r[4:7]))
    metrics.check_fp64(metrics.parity(r[7:], None, ro, lo, so))


@MODES
def test_no_points(saved):
    """m = 0: every node gradient is zero, dL/dx is empty."""
    c = inputs.grad_workload(n=65, m=10)
    nodes, vals = _t(c["nodes"]), _t(c["values"])
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    if saved:
        r, st = fh.eval_forward(nodes, vals, c["d"], x, derivative=saved == "deriv")
        assert r.numel() == 0
        gv, gx, gn = fh.eval_backward_saved(st, x)
    else:
        gv, gx, gn = fh.eval_backward(nodes, vals, c["d"], x, x)
    torch.cuda.synchronize()
    assert gx.numel() == 0
    assert torch.count_nonzero(gv) == 0 and torch.count_nonzero(gn) == 0


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_saved_forward_derivative(precision):
    """With the derivative the forward returns fh_eval_deriv's r and r' bit
    for bit, and dL/dx_p = g_p r'(x_p) exactly (one product)."""
    c = inputs.grad_workload(n=300, m=9001)
    pts = c["points"].copy()
    pts[:2] = c["nodes"][[0, 150]]
    pts[2] = np.nan
    args = (_t(c["nodes"]), _t(c["values"]), c["d"], _t(pts))
    r, st = fh.eval_forward(*args, derivative=True, precision=precision)
    r2, dr2 = fh.eval_deriv(*args, precision=precision)
    for u, v in ((r, r2), (st.dr, dr2)):
        assert torch.equal(torch.isnan(u), torch.isnan(v))
        assert torch.equal(u.nan_to_num(0.0), v.nan_to_num(0.0))
    g = _t(c["grad"])
    gx = fh.eval_backward_saved(st, g, need_values=False, need_nodes=False)[1]
    want = g * dr2
    assert torch.equal(torch.isnan(gx), torch.isnan(want))
    assert torch.equal(gx.nan_to_num(0.0), want.nan_to_num(0.0))
    # binary64: neither r nor the node gradients depend on whether the
    # forward formed r' (split: the node gradients come from the forward's
    # records with r', from the two split passes without)
    if precision == "fp64":
        r0, st0 = fh.eval_forward(*args, precision=precision)
        assert torch.equal(torch.isnan(r0), torch.isnan(r))
        assert torch.equal(r0.nan_to_num(0.0), r.nan_to_num(0.0))
        for u, v in zip(fh.eval_backward_saved(st, g, need_x=False),
                        fh.eval_backward_saved(st0, g, need_x=False)):
            assert (u is None and v is None) or torch.equal(u, v)


def test_saved_forward_bits_of_eval_variant():
    """fh_eval_forward's r has the bits of fh_eval with binary64 launch
    variant 4 (two points per lane, groups of eight, plain sums: the same
    operations in the same order), hits and NaN included."""
    c = inputs.grad_workload(n=777, m=20011)
    pts = c["points"].copy()
    pts[:3] = c["nodes"][[0, 5, 776]]
    pts[3] = np.nan
    args = (_t(c["nodes"]), _t(c["values"]), c["d"], _t(pts))
    r, _ = fh.eval_forward(*args)
    fh.tune_force("fp64", 4)
    try:
        r4 = fh.evaluate(*args)
    finally:
        fh.tune_force("fp64", -1)
    assert torch.equal(torch.isnan(r), torch.isnan(r4))
    assert torch.equal(r.nan_to_num(0.0), r4.nan_to_num(0.0))


@pytest.mark.parametrize("n", [8191, 8193, 9000])
def test_saved_many_node_tiles(n):
    """More node tiles than tile groups (n > 64 tiles of 128 nodes): each
    wave adds the point-side sums of several tiles in place."""
    g = np.random.default_rng(n)
    nodes = inputs.equispaced(n)
    vals = np.sin(7 * nodes) + 0.1 * g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1, 1, 1500), nodes[::1000]])
    grad = g.standard_normal(pts.size)
    _check_against_oracle(nodes, vals, 3, pts, grad, saved="fused")
