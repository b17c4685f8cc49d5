"""Launch variants that take the Lebesgue sum by node blocks (binary64:
blocks of 16 nodes; FP32-split: the 32-node tiles of its binary32 sums).

Floater-Hormann weights alternate in sign, so on a block of nodes that lies
on one side of the point the terms |w_k t_k| alternate like w_k, and one
multiply-add per pair gives both sum_k a_k and sum_k |a_k| (E + O and
|E - O| of the block's even and odd sums).  The block that contains the
point is recomputed exactly after the node loop.  Checked against the
oracle: points in every block, on both sides of every block boundary, next
to the first and last node of a block, outside the nodes, hits, NaN/inf;
caller weights that do not alternate take plain sums; r alone has the bits
of r computed with Lambda."""
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


PRECS = ["fp64", "split"]


def _block_variants(prec):
    return [v for v in fh.variants(prec) if fh.variant_lebesgue_block(prec, v[0]) > 0]


def _plain_twin(prec, p, g, s):
    for vid, vp, vg, vs in fh.variants(prec):
        if (vp, vg, vs) == (p, g, s) and fh.variant_lebesgue_block(prec, vid) == 0:
            return vid
    raise AssertionError("no plain variant with the same shape")


def _check(prec, r, lam, ref):
    r_o, lam_o, s_o = ref
    if prec == "fp64":
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
    else:
        st = metrics.parity(r, lam, r_o, lam_o, s_o, metrics.SPLIT_LAMBDA_MAX)
        metrics.check_split(st)
    return st


def _points(nodes, g, m=20000, u=16):
    n = nodes.size
    gaps = np.diff(nodes)
    b = np.arange(u, n, u)  # first node of every block after the first
    parts = [g.uniform(nodes[0], nodes[-1], m),
             nodes[b - 1] + 0.5 * gaps[b - 1],            # between two blocks
             nodes[b] + 1e-3 * gaps[np.minimum(b, n - 2)],  # just inside a block's first node
             nodes[b - 1] - 1e-3 * gaps[b - 2],             # just inside a block's last node
             nodes[::7],                                    # hits
             [nodes[0] - 0.5, nodes[-1] + 0.5, np.nan, np.inf, -np.inf]]
    return np.concatenate(parts)


def _run(nodes, vals, d, pts, vid, weights=None, lebesgue=True, prec="fp64"):
    fh.tune_force(prec, vid)
    try:
        out = fh.evaluate(_t(nodes), _t(vals), d, _t(pts), lebesgue=lebesgue, precision=prec,
                          weights=None if weights is None else _t(weights))
    finally:
        fh.tune_force(prec, -1)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind,n,d", [("equispaced", 257, 3), ("jittered", 1001, 8),
                                      ("equispaced", 40, 0), ("jittered", 17, 4),
                                      ("cheb2", 129, 2), ("equispaced", 4097, 6)])
def test_block_variants_against_oracle(kind, n, d, prec):
    g = np.random.default_rng(n + d)
    nodes = {"equispaced": inputs.equispaced, "cheb2": inputs.cheb2}.get(
        kind, lambda k: inputs.jittered_nodes(k, g, rel=0.3))(n)
    vals = np.cos(5 * nodes) + 0.1 * g.standard_normal(n)
    pts = _points(nodes, g)
    ref = oracle.evaluate(nodes, vals, d, pts)
    hit = np.isin(pts, nodes)
    variants = _block_variants(prec)
    assert variants
    for vid, p, grp, s in variants:
        r, lam = _run(nodes, vals, d, pts, vid, prec=prec)
        r, lam = r.cpu().numpy(), lam.cpu().numpy()
        st = _check(prec, r, lam, ref)
        if prec == "fp64":
            bound = (n + 33) * U64
            assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)
        assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
        assert np.all(lam[hit] == 1.0), vid


@pytest.mark.parametrize("prec", PRECS)
def test_lebesgue_only_and_r_only(prec):
    g = np.random.default_rng(3)
    nodes = inputs.jittered_nodes(1001, g, rel=0.3)
    vals = g.standard_normal(1001)
    pts = _points(nodes, g)
    _, lam_o, s_o = oracle.evaluate(nodes, vals, 5, pts)
    tol = 1e-13 if prec == "fp64" else 2.0 ** -17
    for vid, p, grp, s in _block_variants(prec):
        fh.tune_force(prec, vid)
        try:
            lam = fh.lebesgue(_t(nodes), 5, _t(pts), precision=prec)
        finally:
            fh.tune_force(prec, -1)
        lam = lam.cpu().numpy()
        fin = np.isfinite(lam_o)
        assert np.array_equal(np.isnan(lam), np.isnan(lam_o))
        assert np.max(np.abs(lam[fin] - lam_o[fin]) / (lam_o[fin] * (1 + lam_o[fin]))) <= tol
        # r alone: the same bits as with Lambda (D is summed by blocks either way)
        r_b = _run(nodes, vals, 5, pts, vid, lebesgue=False, prec=prec)
        r_l, _ = _run(nodes, vals, 5, pts, vid, prec=prec)
        a, b = r_b.cpu().numpy(), r_l.cpu().numpy()
        assert np.array_equal(np.isnan(a), np.isnan(b))
        assert np.array_equal(a[~np.isnan(a)].view(np.uint64), b[~np.isnan(b)].view(np.uint64))


@pytest.mark.parametrize("prec", PRECS)
def test_caller_weights(prec):
    """Caller weights that do not alternate in sign (positive weights, and the
    library's weights with one sign flipped) take plain sums: the block
    variants then give their plain twin's bits.  Caller weights that do
    alternate (the library's own, passed in) take block sums and give the
    bits of the internal weight pass.  Both match the oracle with those
    weights."""
    g = np.random.default_rng(11)
    nodes = inputs.jittered_nodes(513, g, rel=0.3)
    vals = g.standard_normal(513)
    pts = _points(nodes, g, m=5000)
    w_lib = oracle.weights(nodes, 3)
    w_flip = w_lib.copy()
    w_flip[200] = -w_flip[200]
    for w, alternating in ((g.uniform(0.5, 2.0, 513), False), (w_flip, False), (w_lib, True)):
        ref = oracle.evaluate(nodes, vals, 3, pts, w=w)
        for vid, p, grp, s in _block_variants(prec):
            r, lam = _run(nodes, vals, 3, pts, vid, weights=w, prec=prec)
            if alternating:
                r2, lam2 = _run(nodes, vals, 3, pts, vid, prec=prec)
            else:
                r2, lam2 = _run(nodes, vals, 3, pts, _plain_twin(prec, p, grp, s), weights=w,
                                prec=prec)
            for a, b in ((r, r2), (lam, lam2)):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                assert np.array_equal(np.isnan(a), np.isnan(b)), (vid, alternating)
                assert np.array_equal(a[~np.isnan(a)].view(np.uint64),
                                      b[~np.isnan(b)].view(np.uint64)), (vid, alternating)
            _check(prec, r.cpu().numpy(), lam.cpu().numpy(), ref)


def test_prepared_table_switches_between_weight_sources():
    """One workspace prepared alternately with positive caller weights and
    with the library's weights: the flag that selects block sums follows the
    last packing, so every result has the bits of the same call on a fresh
    workspace (plain sums with the caller's weights, block sums without)."""
    g = np.random.default_rng(5)
    nodes = inputs.jittered_nodes(300, g, rel=0.3)
    vals = g.standard_normal(300)
    pts = _points(nodes, g, m=4000)
    w_pos = g.uniform(0.5, 2.0, 300)
    vid = _block_variants("fp64")[0][0]
    fresh = {"caller": _run(nodes, vals, 2, pts, vid, weights=w_pos),
             "library": _run(nodes, vals, 2, pts, vid)}
    ref = {"caller": oracle.evaluate(nodes, vals, 2, pts, w=w_pos),
           "library": oracle.evaluate(nodes, vals, 2, pts)}
    ws = fh.Workspace(DEV, fh.workspace_size(fh.FH_OP_EVAL, 300, pts.size, 2))
    fh.tune_force("fp64", vid)
    try:
        for src in ("caller", "library", "caller", "library"):
            w = _t(w_pos) if src == "caller" else None
            r, lam = fh.evaluate(_t(nodes), _t(vals), 2, _t(pts), lebesgue=True, ws=ws, weights=w)
            torch.cuda.synchronize()
            for a, b in ((r, fresh[src][0]), (lam, fresh[src][1])):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                assert np.array_equal(np.isnan(a), np.isnan(b)), src
                assert np.array_equal(a[~np.isnan(a)].view(np.uint64),
                                      b[~np.isnan(b)].view(np.uint64)), src
            st = metrics.parity(r.cpu().numpy(), lam.cpu().numpy(), *ref[src])
            metrics.check_fp64(st, lam_metric="cond")
    finally:
        fh.tune_force("fp64", -1)
