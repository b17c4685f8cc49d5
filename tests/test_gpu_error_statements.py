"""The stated first-order error bounds of the division-light accumulation.

Binary64 (simultaneous inversion of 4 or 8 differences per reciprocal):
each reciprocal carries at most 27 u (the hardware estimate, at most
2^-24.37, squared by the Newton step, about 21 u, plus the roundings of the
product tree that do not cancel), the difference 1 u and the weighted value
1 u; recursive summation adds at most n u; with the oracle's own 3 u the
computed r and Lambda differ from the oracle's by at most (n + 33) u in
e_cond terms.  The node-pair variants evaluate two terms at once through the
block's coordinates: at a point at least one outer node spacing s from the
block (pair spans at most 8 s and node offsets from the block's anchor at most
16 s, the pack's test) each pair term carries at most about
(32 + 4 * 16 + 9 * 8 / 4) u = 114 u instead of 29 u, so their bound is
(n + 33 + 85) u; the blocks next to the point are summed node by node.
The octet variants sum the blocks far from a point by octets, rational
functions of eight nodes in monomial form, whose terms carry at most about
30 F u + 30 u with the pack's F <= 8 (270 u): their bound is (n + 33 + 245) u.

FP32-split: the float-float difference 2 u32, the reciprocal 2 u32 (one ulp,
G = 1) or 6 u32 (G = 4: the ulp of v_rcp_f32 plus four roundings), the
binary32 weight 1 u32, the 32-term binary32 tile sum 32 u32: at most 41 u32
(G = 4), checked as 44 u32, at points at least 2^-20 from every node (closer
points add the head/tail representation error 2^-47 |x| / |x - x_k| to one
dominant term; the 2^-17 bar of the other tests covers them).
"""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U64, U32 = 2.0 ** -53, 2.0 ** -24


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _case(n, d, m, seed):
    g = np.random.default_rng(seed)
    nodes = inputs.jittered_nodes(n, g, rel=0.3)
    om, amp = inputs.sines_params(g)
    vals = inputs.sines(nodes, om, amp)
    pts = np.concatenate([g.uniform(-1, 1, m), nodes[::max(1, n // 50)]])
    return nodes, vals, d, pts


def _run(nodes, vals, d, pts, precision):
    r, lam = fh.evaluate(_t(nodes), _t(vals), d, _t(pts), lebesgue=True, precision=precision)
    torch.cuda.synchronize()
    return r.cpu().numpy(), lam.cpu().numpy()


@pytest.mark.parametrize("n,d", [(17, 3), (257, 5), (1001, 4), (4097, 6)])
def test_fp64_first_order_bound(n, d):
    nodes, vals, d, pts = _case(n, d, 20000, n)
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    for vid, p, grp, s in fh.variants("fp64"):
        fh.tune_force("fp64", vid)
        try:
            r, lam = _run(nodes, vals, d, pts, "fp64")
        finally:
            fh.tune_force("fp64", -1)
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        extra = 245 if fh.variant_octets("fp64", vid) else (
            85 if fh.variant_node_pairs("fp64", vid) else 0)
        bound = (n + 33 + extra) * U64
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, grp, st)


@pytest.mark.parametrize("n,d", [(64, 3), (1001, 4), (4097, 6)])
def test_split_first_order_bound(n, d):
    nodes, vals, d, pts = _case(n, d, 20000, 7 * n)
    # points at least 2^-20 from every node
    k = np.clip(np.searchsorted(nodes, pts), 1, n - 1)
    gap = np.minimum(np.abs(pts - nodes[k - 1]), np.abs(pts - nodes[k]))
    pts = pts[gap >= 2.0 ** -20]
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    for vid, p, grp, s in fh.variants("split"):
        fh.tune_force("split", vid)
        try:
            r, lam = _run(nodes, vals, d, pts, "split")
        finally:
            fh.tune_force("split", -1)
        st = metrics.parity(r, lam, r_o, lam_o, s_o, metrics.SPLIT_TERMS_LAMBDA_MAX)
        bound = 44 * U32
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, grp, st)
