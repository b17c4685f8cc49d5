"""Group products in the subnormal range.  The binary64 node loops hold no
range test: a zero, infinite or NaN group product makes the refined
reciprocal NaN, and the lane is flagged when its sum D ends up non-finite.
A subnormal product whose estimate overflows is flagged the same way; one
in (2^-1024, 2^-1022) with a finite reciprocal is not, and its rounding
(2^-51 relative instead of 2^-53) adds at most 3.5 u to the terms of its
group.  Sixteen nodes in a cluster so tight that the product of the
differences of one node group falls in that range (spacing 2^-128.5 for
groups of 8, 2^-255.3 for groups of 4) put both cases under test, for every
binary64 launch variant, against the oracle: the binary64 bar, and the
first-order statement (n + 30) u plus the corner's 3.5 u plus the oracle's
3 u."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U64 = 2.0 ** -53
SPACING = {8: 2.0 ** -128.5, 4: 2.0 ** -255.3}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _group_product(x, nodes, g):
    """The first group's product of differences, in the kernels' tree order."""
    d = x[:, None] - nodes[None, :g]
    if g == 8:
        return ((d[:, 0] * d[:, 1]) * (d[:, 2] * d[:, 3])) * ((d[:, 4] * d[:, 5]) * (d[:, 6] * d[:, 7]))
    return (d[:, 0] * d[:, 1]) * (d[:, 2] * d[:, 3])


def _case(g):
    h = SPACING[g]
    nodes = np.arange(16) * h
    rng = np.random.default_rng(1000 + g)
    vals = rng.standard_normal(16)
    pts = np.concatenate([rng.uniform(0.0, (g - 1) * h, 6000),      # first group: tiny products
                          rng.uniform(0.0, 15 * h, 2000),            # anywhere in the cluster
                          nodes[::3],                                # exact hits
                          [-3 * h, 20 * h]])                         # outside
    return nodes, vals, pts


@pytest.mark.parametrize("g", [8, 4])
def test_subnormal_group_products(g):
    nodes, vals, pts = _case(g)
    q = np.abs(_group_product(pts, nodes, g))
    # the case is present: unflagged subnormal products and overflowing ones
    assert np.count_nonzero((q > 2.0 ** -1024) & (q < 2.0 ** -1022)) > 500
    assert np.count_nonzero((q > 0) & (q <= 2.0 ** -1024)) > 100
    d = 2
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    n = nodes.size
    ran = 0
    for vid, p, grp, s in fh.variants("fp64"):
        if grp != g:
            continue
        fh.tune_force("fp64", vid)
        try:
            r, lam = fh.evaluate(_t(nodes), _t(vals), d, _t(pts), lebesgue=True)
        finally:
            fh.tune_force("fp64", -1)
        torch.cuda.synchronize()
        r, lam = r.cpu().numpy(), lam.cpu().numpy()
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
        bound = (n + 30 + 3.5 + 3) * U64
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)
        hit = np.isin(pts, nodes)
        assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
        assert np.all(lam[hit] == 1.0), vid
        ran += 1
    assert ran > 0
