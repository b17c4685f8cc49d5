"""Batched evaluation (fh_batch_create / fh_eval_batched): per-instance parity
with the FP64 oracle, bit-for-bit agreement with the single-interpolant
kernel that runs the same per-point operations, edge instances, graph
replays interleaved with eager work, device status, and the full 4096-
instance workload on sampled instances."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _batch(c, precision="fp64", lebesgue=True):
    b = fh.Batch(c["n"], c["d"], c["m"], _t(c["nodes"]), _t(c["values"]), _t(c["points"]),
                 lebesgue=lebesgue, precision=precision)
    out = b()
    torch.cuda.synchronize()
    return b, out


def _slices(c, i):
    return (slice(int(c["node_off"][i]), int(c["node_off"][i + 1])),
            slice(int(c["pt_off"][i]), int(c["pt_off"][i + 1])))


def _small_batch(salt=0, count=48):
    return inputs.batched_workload(count=count, n_range=(16, 300), m_range=(100, 3000), salt=salt)


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_instances_against_oracle(precision):
    c = _small_batch()
    b, (r, lam) = _batch(c, precision)
    r, lam = r.cpu().numpy(), lam.cpu().numpy()
    for i in range(c["n"].size):
        ns, ps = _slices(c, i)
        r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(c["d"][i]),
                                          c["points"][ps])
        if precision == "fp64":
            metrics.check_fp64(metrics.parity(r[ps], lam[ps], r_o, lam_o, s_o), lam_metric="cond")
        else:
            metrics.check_split(metrics.parity(r[ps], lam[ps], r_o, lam_o, s_o,
                                               metrics.SPLIT_LAMBDA_MAX))
    b.close()


@pytest.mark.parametrize("lebesgue", [True, False])
@pytest.mark.parametrize("precision,single_variant", [("fp64", 4), ("split", 9)])
def test_bitwise_equal_to_single_kernel(precision, single_variant, lebesgue):
    """The batched kernel (2 points per lane) runs, per point, exactly the
    operations of the single-interpolant variant with 2 points per lane and
    no node split (binary64: plain sums; split: sums by node tiles, the
    batch's weights being the library's), so the outputs agree bit for bit,
    with Lambda and for r alone.  The single tables' longer zero-weight
    padding adds exact zeros."""
    c = _small_batch(salt=1, count=16)
    fh.tune_force("batched_" + precision, 1)
    try:
        b, out = _batch(c, precision, lebesgue=lebesgue)
    finally:
        fh.tune_force("batched_" + precision, -1)
    r, lam = out if lebesgue else (out, None)
    fh.tune_force(precision, single_variant)
    try:
        for i in range(c["n"].size):
            ns, ps = _slices(c, i)
            o1 = fh.evaluate(_t(c["nodes"][ns]), _t(c["values"][ns]), int(c["d"][i]),
                             _t(c["points"][ps]), lebesgue=lebesgue, precision=precision)
            r1, l1 = o1 if lebesgue else (o1, None)
            assert torch.equal(r1, r[ps]), i
            if lebesgue:
                assert torch.equal(l1, lam[ps]), i
    finally:
        fh.tune_force(precision, -1)
    b.close()


def _edge_batch():
    g = np.random.default_rng(4)
    specs = [(1, 0, 5), (2, 1, 0), (16, 10, 1), (2048, 1, 700), (17, 3, 257), (300, 0, 513),
             (64, 63, 100), (5, 2, 0)]
    n = np.array([s[0] for s in specs])
    d = np.array([s[1] for s in specs], dtype=np.int32)
    m = np.array([s[2] for s in specs])
    nodes, vals, pts = [], [], []
    for (ni, di, mi) in specs:
        x = inputs.cheb2(ni) if ni > 2 else inputs.equispaced(ni)
        nodes.append(x)
        vals.append(g.standard_normal(ni))
        p = g.uniform(-1, 1, size=mi)
        if mi > 3:
            p[:2] = x[[0, -1]]        # exact hits
        pts.append(p)
    c = {"n": n, "d": d, "m": m, "nodes": np.concatenate(nodes), "values": np.concatenate(vals),
         "points": np.concatenate(pts)}
    c["node_off"] = np.concatenate([[0], np.cumsum(n)])
    c["pt_off"] = np.concatenate([[0], np.cumsum(m)])
    return c


def test_edge_instances():
    c = _edge_batch()
    n, d, m = c["n"], c["d"], c["m"]
    b, (r, lam) = _batch(c)
    r, lam = r.cpu().numpy(), lam.cpu().numpy()
    for i in range(n.size):
        ns, ps = _slices(c, i)
        if m[i] == 0:
            continue
        r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(d[i]),
                                          c["points"][ps])
        metrics.check_fp64(metrics.parity(r[ps], lam[ps], r_o, lam_o, s_o), lam_metric="cond")
        hit = np.isin(c["points"][ps], c["nodes"][ns])
        assert np.array_equal(r[ps][hit], r_o[hit]) and np.all(lam[ps][hit] == 1.0)
    b.close()


def _bit_class(family, vid):
    shape = {v[0]: v[1:] for v in fh.variants(family)}[vid]
    return (shape[1], shape[2], fh.variant_lebesgue_block(family, vid),
            fh.variant_node_pairs(family, vid))


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("lebesgue", [True, False])
def test_every_batched_variant(precision, lebesgue):
    """Every launch variant of the batched kernel (points per lane, node
    split, Lebesgue block, passes per strip), forced one at a time, on edge
    instances (n = 1, 2, 16, ..., m = 0, 1, ragged, exact hits) and a
    seeded small batch: each instance within the oracle's bar, and variants
    that sum in the same order (they differ in points per lane or strip
    length only) give the same bits."""
    family = "batched_" + precision
    c = _edge_batch()
    small = _small_batch(salt=7, count=24)
    bits = {}
    for vid, *_ in fh.variants(family):
        fh.tune_force(family, vid)
        try:
            outs = [_batch(cc, precision, lebesgue=lebesgue) for cc in (c, small)]
        finally:
            fh.tune_force(family, -1)
        for (b, out), cc in zip(outs, (c, small)):
            assert b.variant == vid
            r, lam = out if lebesgue else (out, None)
            r_h = r.cpu().numpy()
            lam_h = lam.cpu().numpy() if lebesgue else None
            for i in range(cc["n"].size):
                ns, ps = _slices(cc, i)
                if ps.stop == ps.start:
                    continue
                r_o, lam_o, s_o = oracle.evaluate(cc["nodes"][ns], cc["values"][ns],
                                                  int(cc["d"][i]), cc["points"][ps])
                st = metrics.parity(r_h[ps], lam_h[ps] if lebesgue else None, r_o, lam_o, s_o,
                                    metrics.FP64_LAMBDA_MAX if precision == "fp64" else
                                    metrics.SPLIT_LAMBDA_MAX)
                if precision == "fp64":
                    metrics.check_fp64(st, lam_metric="cond")
                else:
                    assert st["nan_mismatch_r"] == 0 and st["e_cond_max"] <= metrics.SPLIT_TOL, st
                    if lebesgue:
                        assert st["e_cond_lam_max"] <= metrics.SPLIT_TOL, st
                hit = np.isin(cc["points"][ps], cc["nodes"][ns])
                assert np.array_equal(r_h[ps][hit], r_o[hit]), (vid, i)
            b.close()
        key = _bit_class(family, vid)
        got = [o[1] if not lebesgue else torch.cat(o[1]) for o in outs]
        if key in bits:
            assert all(torch.equal(a, b_) for a, b_ in zip(got, bits[key])), (vid, key)
        else:
            bits[key] = got


def test_split_instances_outside_binary32_domain():
    """Instances whose data leave the binary32 domain (values spanning more
    than 2^100, points beyond one span outside the nodes) next to ordinary
    ones and to tiny values that only need their own scale: every instance
    within the split bar, the out-of-domain ones at binary64 accuracy."""
    g = np.random.default_rng(21)
    specs = []   # (nodes, values, d, points, binary64 expected)
    x = inputs.equispaced(200)
    specs.append((x, g.standard_normal(200), 3, g.uniform(-1, 1, 900), False))
    specs.append((x, np.exp(-400.0 * x ** 2), 3, g.uniform(-1, 1, 800), True))
    specs.append((x, 1e-35 * g.standard_normal(200), 3, g.uniform(-1, 1, 600), False))
    specs.append((x, g.standard_normal(200), 3, 3.5 + g.uniform(0, 2.5, 500), True))
    n = np.array([s[0].size for s in specs])
    c = {"n": n, "d": np.array([s[2] for s in specs], dtype=np.int32),
         "m": np.array([s[3].size for s in specs]),
         "nodes": np.concatenate([s[0] for s in specs]),
         "values": np.concatenate([s[1] for s in specs]),
         "points": np.concatenate([s[3] for s in specs])}
    c["node_off"] = np.concatenate([[0], np.cumsum(c["n"])])
    c["pt_off"] = np.concatenate([[0], np.cumsum(c["m"])])
    b, (r, lam) = _batch(c, "split")
    r, lam = r.cpu().numpy(), lam.cpu().numpy()
    for i, s in enumerate(specs):
        ns, ps = _slices(c, i)
        r_o, lam_o, s_o = oracle.evaluate(s[0], s[1], s[2], s[3])
        st = metrics.parity(r[ps], lam[ps], r_o, lam_o, s_o, metrics.SPLIT_LAMBDA_MAX)
        metrics.check_split(st)
        if s[4]:
            assert st["e_cond_max"] <= metrics.FP64_TOL, (i, st)
        else:
            assert st["e_cond_max"] > metrics.FP64_TOL, (i, st)
    b.close()


def test_graph_replays_with_eager_work_between():
    c = _small_batch(salt=2)
    b, (r, lam) = _batch(c)
    ref_r, ref_l = r.clone(), lam.clone()
    for k in range(4):
        r.fill_(np.nan)                     # eager work on the same buffers
        junk = torch.randn(1 << 20, device=DEV).sum()  # unrelated eager kernels
        torch.cuda.synchronize()
        b()
        torch.cuda.synchronize()
        assert torch.equal(r, ref_r) and torch.equal(lam, ref_l), k
        assert torch.isfinite(junk)
    b.close()


def test_value_only_and_lebesgue_only():
    c = _small_batch(salt=3, count=12)
    b_full, (r, lam) = _batch(c)
    b_r = fh.Batch(c["n"], c["d"], c["m"], _t(c["nodes"]), _t(c["values"]), _t(c["points"]))
    r2 = b_r()
    b_l = fh.Batch(c["n"], c["d"], c["m"], _t(c["nodes"]), _t(c["values"]), _t(c["points"]),
                   want_r=False, lebesgue=True)
    l2 = b_l()
    torch.cuda.synchronize()
    assert torch.equal(r, r2) and torch.equal(lam, l2)
    for b in (b_full, b_r, b_l):
        b.close()


def test_device_status_for_bad_nodes():
    c = _small_batch(salt=5, count=6)
    nodes = c["nodes"].copy()
    o = int(c["node_off"][3])
    nodes[o + 4] = nodes[o + 3]              # repeated node in instance 3
    c2 = dict(c, nodes=nodes)
    b, _ = _batch(c2)
    st, bits = b.status()
    assert st == fh.FH_E_NODES and bits & 0x1
    st, bits = b.status()
    assert st == fh.FH_OK and bits == 0
    b.close()


def test_bad_batch_arguments():
    with pytest.raises(fh.FhError) as e:
        fh.Batch([5, 4], [5, 1], [10, 10], _t(np.linspace(-1, 1, 9)), _t(np.zeros(9)),
                 _t(np.zeros(20)))
    assert e.value.code == fh.FH_E_DEGREE
    with pytest.raises(ValueError):
        fh.Batch([5], [1], [10], _t(np.linspace(-1, 1, 4)), _t(np.zeros(4)), _t(np.zeros(10)))


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_full_workload_sampled(precision):
    """All 4096 instances (about 2e8 points) in one launch, in the variant
    the tuner's table gives that shape; 24 seeded instances checked against
    the oracle on up to 1500 points each: the first-order bars up to
    Lambda = 2^40, the Lambda-scaled bars up to 2^48, and how many sampled
    points lie beyond 2^48 (no correct digits on either side) is bounded --
    about 6.5 % of the workload's points, by a sample of 60 instances.  The
    split kernel's conditioning guard sends every point it cannot trust to
    binary64, so both precisions are held to the same bands."""
    c = inputs.batched_workload()
    b, (r, lam) = _batch(c, precision)
    g = np.random.default_rng(9)
    counts = {"n": 0, "n_beyond_lam_max": 0, "n_lambda_scaled": 0, "n_beyond_lam_cap": 0}
    for i in g.choice(c["n"].size, 24, replace=False):
        ns, ps = _slices(c, i)
        sel = np.arange(ps.start, ps.stop)
        sel = sel[g.choice(sel.size, min(1500, sel.size), replace=False)]
        r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(c["d"][i]),
                                          c["points"][sel])
        idx = torch.from_numpy(sel).to(DEV)
        st = metrics.parity(r[idx].cpu().numpy(), lam[idx].cpu().numpy(), r_o, lam_o, s_o,
                            metrics.FP64_LAMBDA_MAX if precision == "fp64" else
                            metrics.SPLIT_LAMBDA_MAX)
        if precision == "fp64":
            metrics.check_fp64(st, lam_metric="cond")
        else:
            metrics.check_split(st)
        counts["n"] += sel.size
        for k in ("n_beyond_lam_max", "n_lambda_scaled", "n_beyond_lam_cap"):
            counts[k] += st[k]
    b.close()
    assert counts["n_lambda_scaled"] > 0, counts          # the scaled band was exercised
    assert counts["n_beyond_lam_cap"] <= 0.12 * counts["n"], counts


@pytest.mark.parametrize("lebesgue", [True, False])
def test_split_batch_ill_conditioned_instances(lebesgue):
    """A split batch mixing instances too ill-conditioned for binary32 terms
    (Chebyshev nodes with d = 8..10: Lebesgue functions up to 1e18) with
    well-conditioned ones: the packing marks the former, whose points then
    all take binary64 terms (the bits of binary64 launch variant 0), while
    the others stay on the binary32 path; every instance within the split
    bar's bands."""
    g = np.random.default_rng(31)
    specs = [(inputs.cheb2(600), 10), (inputs.equispaced(300), 3), (inputs.cheb2(1000), 8),
             (inputs.jittered_nodes(513, g), 4), (inputs.cheb2(129), 9)]
    vals = [g.standard_normal(x.size) for x, _ in specs]
    pts = [g.uniform(-1, 1, 3000 + 17 * i) for i in range(len(specs))]
    c = {"n": np.array([x.size for x, _ in specs]), "d": np.array([d for _, d in specs], np.int32),
         "m": np.array([p.size for p in pts]), "nodes": np.concatenate([x for x, _ in specs]),
         "values": np.concatenate(vals), "points": np.concatenate(pts)}
    c["node_off"] = np.concatenate([[0], np.cumsum(c["n"])])
    c["pt_off"] = np.concatenate([[0], np.cumsum(c["m"])])
    b, out = _batch(c, "split", lebesgue=lebesgue)
    r, lam = out if lebesgue else (out, None)
    r = r.cpu().numpy()
    fh.tune_force("fp64", 0)
    try:
        for i, (x, d) in enumerate(specs):
            ns, ps = _slices(c, i)
            o = fh.evaluate(_t(x), _t(vals[i]), d, _t(pts[i]), lebesgue=lebesgue)
            r64 = (o[0] if lebesgue else o).cpu().numpy()
            r_o, lam_o, s_o = oracle.evaluate(x, vals[i], d, pts[i])
            st = metrics.parity(r[ps], lam[ps].cpu().numpy() if lebesgue else None, r_o, lam_o,
                                s_o, metrics.SPLIT_LAMBDA_MAX)
            assert st["nan_mismatch_r"] == 0 and st["e_cond_max"] <= metrics.SPLIT_TOL, (i, st)
            assert st["e_cond_scaled_max"] <= metrics.SPLIT_TOL, (i, st)
            if np.max(lam_o) > 2.0 ** 20:          # ill-conditioned: binary64 for all points
                assert np.array_equal(r[ps].view(np.int64), r64.view(np.int64)), i
            elif np.max(lam_o) < 2.0 ** 8:         # well-conditioned: binary32 terms
                assert not np.array_equal(r[ps], r64), i
    finally:
        fh.tune_force("fp64", -1)
    b.close()


def test_pair_variants_with_failing_blocks():
    """Binary64 pair variants: in an instance with a block too wide next to
    the node spacings around it (one block stretched 20 times) the loop sums
    that block node by node and the others by pairs, inside the same launch;
    every instance within the oracle's bar and the pair variants' bound, and
    every instance, the stretched ones too, takes the pair sums (bits other
    than the node-block variant's of the same shape)."""
    g = np.random.default_rng(31)
    h = np.ones(199)
    h[48:63] = 20.0
    wide = -1.0 + 2.0 * np.concatenate([[0.0], np.cumsum(h)]) / (1.0 + h.sum())
    specs = [(wide, 3), (inputs.equispaced(300), 4), (inputs.cheb2(129), 2), (wide, 5)]
    n = np.array([x.size for x, _ in specs])
    d = np.array([dd for _, dd in specs], dtype=np.int32)
    m = np.array([1500, 1200, 900, 700])
    pts = [np.concatenate([x[::5], g.uniform(-1, 1, int(mi) - x[::5].size)])
           for (x, _), mi in zip(specs, m)]
    c = {"n": n, "d": d, "m": m, "nodes": np.concatenate([x for x, _ in specs]),
         "values": np.concatenate([np.cos(3 * x) for x, _ in specs]),
         "points": np.concatenate(pts)}
    c["node_off"] = np.concatenate([[0], np.cumsum(n)])
    c["pt_off"] = np.concatenate([[0], np.cumsum(m)])
    shapes = {v[0]: v[1:] for v in fh.variants("batched_fp64")}
    strips = {v: fh.variant_strip_points("batched_fp64", v) for v in shapes}
    pair_ids = [v for v in shapes if fh.variant_node_pairs("batched_fp64", v)]
    assert pair_ids
    for vid in pair_ids:
        twin = next(t for t in shapes if shapes[t] == shapes[vid] and strips[t] == strips[vid]
                    and fh.variant_lebesgue_block("batched_fp64", t) == 16
                    and not fh.variant_node_pairs("batched_fp64", t))
        outs = {}
        for v in (vid, twin):
            fh.tune_force("batched_fp64", v)
            try:
                b, (r, lam) = _batch(c)
            finally:
                fh.tune_force("batched_fp64", -1)
            outs[v] = (r.cpu().numpy(), lam.cpu().numpy())
            b.close()
        r, lam = outs[vid]
        for i in range(n.size):
            ns, ps = _slices(c, i)
            r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(d[i]),
                                              c["points"][ps])
            st = metrics.parity(r[ps], lam[ps], r_o, lam_o, s_o)
            metrics.check_fp64(st, lam_metric="cond")
            bound = (int(n[i]) + 33 + 85) * 2.0 ** -53
            assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, i, st)
            assert not np.array_equal(r[ps], outs[twin][0][ps]), (vid, twin, i)
