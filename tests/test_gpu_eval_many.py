"""Several prepared tables evaluated in one launch (fh_eval_prepared_many):
every table's r and Lambda have the bits of its own fh_eval_prepared call
-- with the tuner's own choices (the launch takes the variant tuned for all
its points only where that sums in the same order as the single call's),
and with one launch variant forced -- for
several launch variants (plain sums, Lebesgue blocks, node splits 2 and 4),
ragged point counts, r alone, Lambda alone, up to 16 tables, tables packed
by fh_prepare_many or one by one; and the oracle's bar on the sines
workload's degree sweep."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _bits_equal(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
        a[~np.isnan(a)].view(np.uint64), b[~np.isnan(b)].view(np.uint64))


def _case(n, m, seed):
    g = np.random.default_rng(seed)
    nodes = inputs.jittered_nodes(n, g, rel=0.3)
    vals = np.sin(4 * nodes) + 0.1 * g.standard_normal(n)
    pts = np.concatenate([g.uniform(nodes[0] - 0.1, nodes[-1] + 0.1, m), nodes[::5],
                          [np.nan, np.inf]])
    return nodes, vals, pts


@pytest.mark.parametrize("n,m,K", [(21, 10021, 3), (1001, 20011, 9), (1001, 1_000_000, 9),
                                   (257, 300_000, 16), (4097, 99_999, 2)])
def test_bits_independent_of_call_shape(n, m, K):
    """No variant forced: each table of one launch over K tables equals its
    own fh_eval_prepared call with the same m, bit for bit."""
    nodes, vals, pts = _case(n, m, 5)
    degrees = [k % min(n, 9) for k in range(K)]
    preps = fh.prepare_many(_t(nodes), _t(vals), degrees)
    x = _t(pts)
    many = fh.eval_many(preps, x, lebesgue=True)
    for c, p in enumerate(preps):
        r1, l1 = p(x, lebesgue=True)
        assert _bits_equal(many[0][c], r1) and _bits_equal(many[1][c], l1), (n, m, K, c)


@pytest.mark.parametrize("vid", [3, 10, 15, 17, 18, 20, 22, 25])
@pytest.mark.parametrize("mode", ["both", "r", "lambda"])
def test_bits_of_single_calls(vid, mode):
    nodes, vals, pts = _case(1001, 20011, 7)
    degrees = list(range(9))
    preps = fh.prepare_many(_t(nodes), _t(vals), degrees)
    x = _t(pts)
    want_r, leb = mode != "lambda", mode != "r"
    fh.tune_force("fp64", vid)
    try:
        many = fh.eval_many(preps, x, want_r=want_r, lebesgue=leb)
        single = [p(x, want_r=want_r, lebesgue=leb) for p in preps]
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    if mode == "both":
        for c in range(len(degrees)):
            assert _bits_equal(many[0][c], single[c][0]), (vid, c)
            assert _bits_equal(many[1][c], single[c][1]), (vid, c)
    else:
        for c in range(len(degrees)):
            assert _bits_equal(many[c], single[c]), (vid, mode, c)


@pytest.mark.parametrize("K,m", [(1, 1), (2, 255), (5, 64 * 37 + 3), (16, 4099)])
def test_counts_and_one_by_one_tables(K, m):
    nodes, vals, pts = _case(129, m, 100 + K)
    degrees = [int(d) for d in np.random.default_rng(K).integers(0, 12, K)]
    preps = [fh.Prepared(_t(nodes), _t(vals), d) for d in degrees]
    x = _t(pts)
    fh.tune_force("fp64", 16)
    try:
        r, lam = fh.eval_many(preps, x, lebesgue=True)
        single = [p(x, lebesgue=True) for p in preps]
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    for c, p in enumerate(preps):
        r1, l1 = single[c]
        assert _bits_equal(r[c], r1) and _bits_equal(lam[c], l1), c
        ro, lo, so = oracle.evaluate(nodes, vals, degrees[c], pts)
        metrics.check_fp64(metrics.parity(r[c].cpu().numpy(), lam[c].cpu().numpy(), ro, lo, so),
                           lam_metric="cond")


@pytest.mark.parametrize("vid", [17, 22, 25])
def test_caller_weights_table_among_library_tables(vid):
    """A table prepared with caller weights that do not alternate takes
    plain sums inside the same launch as block-sum (17) or node-pair (22)
    tables."""
    nodes, vals, pts = _case(300, 5000, 3)
    w_pos = np.random.default_rng(2).uniform(0.5, 2.0, 300)
    preps = [fh.Prepared(_t(nodes), _t(vals), 3),
             fh.Prepared(_t(nodes), _t(vals), 3, weights=_t(w_pos)),
             fh.Prepared(_t(nodes), _t(vals), 5)]
    x = _t(pts)
    fh.tune_force("fp64", vid)
    try:
        r, lam = fh.eval_many(preps, x, lebesgue=True)
        single = [p(x, lebesgue=True) for p in preps]
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    for c in range(3):
        assert _bits_equal(r[c], single[c][0]) and _bits_equal(lam[c], single[c][1]), c
    ro, lo, so = oracle.evaluate(nodes, vals, 3, pts, w=w_pos)
    metrics.check_fp64(metrics.parity(r[1].cpu().numpy(), lam[1].cpu().numpy(), ro, lo, so),
                       lam_metric="cond")


def test_tuned_variant_meets_the_oracle_bar():
    """Untuned calls: the launch picks its variant for K * m points (which
    may differ from a single call's); every table meets the oracle's bar."""
    nodes, vals, pts = _case(21, 10000, 9)
    preps = fh.prepare_many(_t(nodes), _t(vals), [0, 2, 3])
    r, lam = fh.eval_many(preps, _t(pts), lebesgue=True)
    torch.cuda.synchronize()
    for c, d in enumerate([0, 2, 3]):
        ro, lo, so = oracle.evaluate(nodes, vals, d, pts)
        metrics.check_fp64(metrics.parity(r[c].cpu().numpy(), lam[c].cpu().numpy(), ro, lo, so),
                           lam_metric="cond")


def test_sines_sweep_against_oracle_sample():
    """The benchmark's timed path (nine degrees of the full workload in one
    launch, the launch variant the benchmark uses) against the oracle on a
    seeded sample, with the workload bar for Lambda (plain relative error:
    the sweep's Lebesgue functions stay below 200)."""
    c = inputs.sines_workload()
    nodes, vals, pts = c["nodes"], c["values"], c["points"]
    preps = fh.prepare_many(_t(nodes), _t(vals), c["degrees"])
    r, lam = fh.eval_many(preps, _t(pts), lebesgue=True)
    torch.cuda.synchronize()
    sel = np.random.default_rng(0).choice(pts.size, 3000, replace=False)
    for i, d in enumerate(c["degrees"]):
        ro, lo, so = oracle.evaluate(nodes, vals, d, pts[sel])
        st = metrics.parity(r[i].cpu().numpy()[sel], lam[i].cpu().numpy()[sel], ro, lo, so)
        metrics.check_fp64(st, lam_metric="rel")
        assert st["n_beyond_lam_max"] == 0, st


def test_shape_checks():
    nodes, vals, pts = _case(64, 100, 1)
    a = fh.Prepared(_t(nodes), _t(vals), 2)
    b = fh.Prepared(_t(nodes[:-1]), _t(vals[:-1]), 2)
    with pytest.raises(ValueError):
        fh.eval_many([a, b], _t(pts))
    with pytest.raises(ValueError):
        fh.eval_many([a], _t(pts), out=torch.empty((2, pts.size), dtype=torch.float64,
                                                   device=DEV))
    with pytest.raises(fh.FhError):
        fh.eval_many([a] * 17, _t(pts), lebesgue=True)
