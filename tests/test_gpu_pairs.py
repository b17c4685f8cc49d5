"""The node-pair launch variants of the binary64 evaluation.

Two records (a, a+2) of a 16-node block give one rational term
(B x'' + J) / (x''^2 - hh^2) for w_a/(x - x_a) + w_{a+2}/(x - x_{a+2})
(and C, K for the weighted values), with x'' measured from the block's
anchor and the pair's midpoint.  The blocks holding the nodes next to a
point (one, or two for a point between blocks) are masked out of the loop
and summed node by node; a block too wide next to the node spacings around
it (the pack's test) is summed node by node inside the loop, the other
blocks of its table still by pairs.  Checked against the oracle at the
points where the masking decides (every node, one ulp on either side of the
nodes at the block edges, midpoints between blocks, just outside the end
nodes, far away), on tables whose blocks all pass and on tables with
failing blocks (Chebyshev nodes whose last node starts a block of its own,
strongly jittered nodes, a stretched block).
"""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U64 = 2.0 ** -53


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _pair_variants():
    return [v for v in fh.variants("fp64") if fh.variant_node_pairs("fp64", v[0])]


def _bound(vid, n):
    """First-order e_cond bound of a pair variant: (n + 33 + 85) u, and
    (n + 33 + 245) u where the blocks far from the point take octets."""
    return (n + 33 + (245 if fh.variant_octets("fp64", vid) else 85)) * U64


def _run(nodes, vals, d, pts, vid, lebesgue=True):
    fh.tune_force("fp64", vid)
    try:
        out = fh.evaluate(_t(nodes), _t(vals), d, _t(pts), lebesgue=lebesgue)
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    return out


def _edge_points(nodes):
    n = nodes.size
    edges = sorted({k for b in range(0, n, 16) for k in (b - 1, b, b + 15, b + 16) if 0 <= k < n})
    e = nodes[edges]
    gaps = np.diff(nodes)
    mids = nodes[:-1] + 0.5 * gaps
    return np.concatenate([
        nodes,                                           # every node: hits
        np.nextafter(e, np.inf), np.nextafter(e, -np.inf),  # one ulp beside the block edges
        mids[[k for k in edges if k < n - 1]],           # between the edge nodes
        [nodes[0] - 1e-9, nodes[-1] + 1e-9, nodes[0] - 0.3, nodes[-1] + 0.3, -10.0, 1e6],
        [np.nan, np.inf, -np.inf]])


@pytest.mark.parametrize("kind,n,d", [("equispaced", 257, 3), ("cheb2", 300, 5),
                                      ("jittered", 1001, 8), ("equispaced", 17, 2),
                                      ("jittered", 33, 4), ("equispaced", 4, 1)])
def test_block_edges_against_oracle(kind, n, d):
    g = np.random.default_rng(n + 7 * d)
    nodes = {"equispaced": inputs.equispaced, "cheb2": inputs.cheb2}.get(
        kind, lambda k: inputs.jittered_nodes(k, g, rel=0.3))(n)
    vals = np.sin(3 * nodes) + 0.1 * g.standard_normal(n)
    pts = np.concatenate([_edge_points(nodes), g.uniform(nodes[0], nodes[-1], 5000)])
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    hit = np.isin(pts, nodes)
    for vid, p, grp, s in _pair_variants():
        r, lam = _run(nodes, vals, d, pts, vid)
        r, lam = r.cpu().numpy(), lam.cpu().numpy()
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
        bound = _bound(vid, n)
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)
        assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
        assert np.all(lam[hit] == 1.0), vid
        assert np.array_equal(np.isnan(r), np.isnan(r_o)), vid


def _wide_block_nodes(n):
    """Equispaced nodes whose fourth block is stretched 20 times: its pair
    spans are 40 times the spacing just outside it."""
    h = np.ones(n - 1)
    h[48:63] = 20.0
    x = np.concatenate([[0.0], np.cumsum(h)])
    return -1.0 + 2.0 * x / x[-1]


def _failing_blocks(nodes):
    """The blocks of 16 nodes that fail the pack's test, restated on the
    host: pair spans (x_{k+2} - x_k) at most 8 and distances from the
    block's anchor (the midpoint of its first and last record) at most 16
    times the smaller node spacing just outside the block; records beyond
    the last node repeat it; a block with no spacing outside it fails."""
    n = nodes.size
    out = []
    for k0 in range(0, n, 16):
        xs = nodes[np.minimum(np.arange(k0, k0 + 16), n - 1)]
        c = 0.5 * (xs[0] + xs[15])
        ext = np.abs(xs - c).max()
        span = (xs[2:] - xs[:-2]).max()
        sl = nodes[k0] - nodes[k0 - 1] if k0 >= 1 else np.inf
        sr = nodes[k0 + 16] - nodes[k0 + 15] if k0 + 16 < n else np.inf
        so = min(sl, sr)
        if not (so < np.inf and span <= 8 * so and ext <= 16 * so):
            out.append(k0 // 16)
    return out


@pytest.mark.parametrize("kind,n,d", [("cheb2", 4097, 3), ("cheb2", 1025, 6),
                                      ("jittered", 4097, 5), ("wide", 200, 3)])
def test_tables_with_failing_blocks(kind, n, d):
    """The failing blocks are summed node by node inside the pair loop and
    every other block by pairs: within the pair variants' bound at the
    block edges, hits and random points, with hits exact, and with bits
    that differ from the node-block variant's (the passing blocks still take
    pairs)."""
    g = np.random.default_rng(5)
    nodes = {"cheb2": inputs.cheb2, "wide": _wide_block_nodes}.get(
        kind, lambda k: inputs.jittered_nodes(k, g, rel=0.3))(n)
    failing = _failing_blocks(nodes)
    assert failing and len(failing) < (n + 15) // 16, failing
    vals = np.cos(2 * nodes) + 0.1 * g.standard_normal(n)
    pts = np.concatenate([_edge_points(nodes), g.uniform(-1, 1, 4000)])
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    hit = np.isin(pts, nodes)
    for vid, *_ in _pair_variants():
        r, lam = _run(nodes, vals, d, pts, vid)
        r, lam = r.cpu().numpy(), lam.cpu().numpy()
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
        bound = _bound(vid, n)
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)
        assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
        assert np.all(lam[hit] == 1.0), vid
    r22, _ = _run(nodes, vals, d, pts, 22)
    r18, _ = _run(nodes, vals, d, pts, 18)
    assert not torch.equal(r22, r18)


def test_pairs_change_the_bits_of_a_passing_table():
    """On a table that passes the test the pair variants do take the pair
    path: their bits differ from the node-block twin's (the same sums in
    another order), both within the oracle's bar."""
    g = np.random.default_rng(4)
    nodes = inputs.equispaced(513)
    vals = g.standard_normal(513)
    pts = g.uniform(-1, 1, 20000)
    r1, _ = _run(nodes, vals, 4, pts, 22)
    r2, _ = _run(nodes, vals, 4, pts, 18)
    assert not torch.isnan(r1).any() and not torch.equal(r1, r2)


def test_lebesgue_only_and_r_only_bits():
    g = np.random.default_rng(6)
    nodes = inputs.jittered_nodes(700, g, rel=0.3)
    vals = g.standard_normal(700)
    pts = np.concatenate([_edge_points(nodes), g.uniform(-1, 1, 3000)])
    for vid, *_ in _pair_variants():
        r, lam = _run(nodes, vals, 5, pts, vid)
        r_only = _run(nodes, vals, 5, pts, vid, lebesgue=False)
        fh.tune_force("fp64", vid)
        try:
            lam_only = fh.lebesgue(_t(nodes), 5, _t(pts))
        finally:
            fh.tune_force("fp64", -1)
        for a, b in ((r, r_only), (lam, lam_only)):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(np.isnan(a), np.isnan(b)), vid
            assert np.array_equal(a[~np.isnan(a)].view(np.uint64),
                                  b[~np.isnan(b)].view(np.uint64)), vid


def _stretched(n, factor, block=3):
    """Unit node spacing except inside one block, whose internal spacing is
    `factor` times larger: its half-extent is about 7.5 * factor outer
    spacings (the pack's limit is 16), its pair spans 2 * factor."""
    h = np.ones(n - 1)
    h[16 * block:16 * block + 15] = factor
    x = np.concatenate([[0.0], np.cumsum(h)])
    return -1.0 + 2.0 * x / x[-1]


@pytest.mark.parametrize("factor,passes", [(2.1, True), (2.2, False)])
def test_block_at_the_width_limit(factor, passes):
    """A block just inside (half-extent 15.75 outer spacings) and just
    outside (16.5) the pack's limit: inside, the pair sums are used on it,
    outside, it is summed node by node; either way the points nearest to the
    block that it does not mask (one outer spacing away, and one ulp closer)
    meet the pair variants' bound."""
    g = np.random.default_rng(12)
    n, d = 160, 4
    nodes = _stretched(n, factor)
    assert (_failing_blocks(nodes) == [3]) != passes
    vals = np.sin(4 * nodes) + 0.05 * g.standard_normal(n)
    b0, b1 = 48, 63  # the stretched block's first and last node
    near = []
    for k in (b0 - 1, b1 + 1):  # the nodes just outside it
        for t in (1e-9, 1e-3, 0.25, 0.5, 0.75, 1 - 1e-3):
            near += [nodes[k - 1] + t * (nodes[k] - nodes[k - 1]),
                     nodes[k] + t * (nodes[k + 1] - nodes[k])]
    near = np.array(near)
    pts = np.concatenate([near, np.nextafter(near, np.inf), np.nextafter(near, -np.inf),
                          _edge_points(nodes), g.uniform(-1, 1, 3000)])
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    for vid, *_ in _pair_variants():
        r, lam = _run(nodes, vals, d, pts, vid)
        st = metrics.parity(r.cpu().numpy(), lam.cpu().numpy(), r_o, lam_o, s_o)
        bound = _bound(vid, n)
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)


@pytest.mark.parametrize("scale", [1e-7, 1e7, 1e-60, 1e60])
def test_scaled_spans(scale):
    """Node spans far from 1: the block coordinates scale with the nodes,
    and spans whose pair denominators leave the binary64 range send the
    points to the exact branch; either way within the oracle's bar."""
    g = np.random.default_rng(13)
    nodes = inputs.equispaced(257) * scale
    vals = g.standard_normal(257)
    pts = np.concatenate([g.uniform(-1, 1, 4000) * scale, nodes[::9],
                          np.nextafter(nodes[16::16], np.inf)])
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, 3, pts)
    for vid, *_ in _pair_variants():
        r, lam = _run(nodes, vals, 3, pts, vid)
        st = metrics.parity(r.cpu().numpy(), lam.cpu().numpy(), r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
        bound = _bound(vid, 257)
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, scale, st)
