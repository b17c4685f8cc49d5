"""The octet launch variants of the binary64 evaluation (25, 26).

The blocks far from a point -- at least two whole blocks beyond the blocks
of its neighbouring nodes -- are summed by octets, the eight even and the
eight odd records of a block each as one rational function in monomial
form; the launch sorts the points by node block first, so that most blocks
serve every point of a wave, and writes each result to the point's original
position.  Checked against the oracle within the octet variants' bound, and
bit for bit: a point's result does not depend on the other points (subsets,
orders, duplicates), a workspace without room for the sorted points and a
table that fails the octet test give the pair variant of the same shape,
and a launch over several tables gives each the bits of its own call, also
when the tables' nodes differ."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U64 = 2.0 ** -53
TWIN = {25: 22, 26: 20}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _run(nodes, vals, d, pts, vid, lebesgue=True, ws_m=None):
    """fh_eval under a forced variant, r and Lambda, with a workspace of
    fh_workspace_size(FH_OP_EVAL, n, ws_m, d) bytes (default ws_m: the point
    count)."""
    n, m = nodes.size, len(pts)
    nbytes = fh.workspace_size(fh.FH_OP_EVAL, n, m if ws_m is None else ws_m, d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    ws[:256].zero_()
    xn, f, x = _t(nodes), _t(vals), _t(pts)
    r = torch.empty(m, dtype=torch.float64, device=DEV)
    lam = torch.empty_like(r) if lebesgue else None
    fh.tune_force("fp64", vid)
    try:
        st = fh.load().fh_eval(fh._ptr(xn), fh._ptr(f), n, d, fh._ptr(x), m, fh._ptr(r),
                               fh._ptr(lam), None, fh.FH_FP64, fh._ptr(ws), nbytes,
                               fh._stream(torch.device(DEV)))
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    assert st == 0, st
    return (r, lam) if lebesgue else r


def _bits(a):
    a = a.cpu().numpy()
    return np.where(np.isnan(a), np.nan, a).view(np.uint64)


def _served_edges(nodes):
    """Midpoints just beyond the closest points each block's octets serve
    (L = x_{16b-33}, R = x_{16b+48}): where the octets' error factor is
    largest."""
    n = nodes.size
    out = []
    for k0 in range(0, n, 16):
        kl, kr = k0 - 33, k0 + 48
        if kl >= 1:
            out.append(nodes[kl] - 0.5 * (nodes[kl] - nodes[kl - 1]))
        if kr + 1 < n:
            out.append(nodes[kr] + 0.5 * (nodes[kr + 1] - nodes[kr]))
    return np.array(out)


def _points(nodes, g, m):
    n = nodes.size
    e = nodes[sorted({k for b in range(0, n, 16) for k in (b - 1, b, b + 15, b + 16)
                      if 0 <= k < n})]
    return np.concatenate([nodes, _served_edges(nodes), np.nextafter(e, np.inf),
                           np.nextafter(e, -np.inf),
                           0.5 * (nodes[:-1] + nodes[1:]),
                           [nodes[0] - 1e-9, nodes[-1] + 1e-9, -3.0, 5.0, np.nan, np.inf],
                           g.uniform(nodes[0], nodes[-1], m)])


@pytest.mark.parametrize("kind,n,d", [("equispaced", 1001, 8), ("cheb2", 1025, 3),
                                      ("jittered", 4097, 5), ("equispaced", 257, 4),
                                      ("equispaced", 40, 3)])
def test_against_oracle(kind, n, d):
    g = np.random.default_rng(n + d)
    nodes = {"equispaced": inputs.equispaced, "cheb2": inputs.cheb2}.get(
        kind, lambda k: inputs.jittered_nodes(k, g, rel=0.3))(n)
    vals = np.sin(3 * nodes) + 0.1 * g.standard_normal(n)
    pts = _points(nodes, g, 20000)
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts)
    hit = np.isin(pts, nodes)
    bound = (n + 33 + 240) * U64
    for vid in (25, 26):
        r, lam = _run(nodes, vals, d, pts, vid)
        r, lam = r.cpu().numpy(), lam.cpu().numpy()
        st = metrics.parity(r, lam, r_o, lam_o, s_o)
        metrics.check_fp64(st, lam_metric="cond")
        assert st["e_cond_max"] <= bound and st["e_cond_lam_max"] <= bound, (vid, st)
        assert np.array_equal(r[hit], vals[np.searchsorted(nodes, pts[hit])]), vid
        assert np.all(lam[hit] == 1.0), vid
        assert np.array_equal(np.isnan(r), np.isnan(r_o)), vid


def test_bits_do_not_depend_on_the_other_points():
    """Subsets, reversed and sorted orders and repeated points: each point
    gets the same bits (the form a block takes for a point depends on the
    point and the table only)."""
    g = np.random.default_rng(7)
    nodes = inputs.equispaced(1001)
    vals = g.standard_normal(1001)
    pts = g.uniform(-1, 1, 200000)
    r, lam = _run(nodes, vals, 6, pts, 25)
    for sel in (np.arange(0, 200000, 13)[::-1], np.argsort(pts), np.repeat(np.arange(50), 1000),
                np.arange(7)):
        r2, lam2 = _run(nodes, vals, 6, pts[sel], 25)
        assert np.array_equal(_bits(r2), _bits(r)[sel]) and np.array_equal(_bits(lam2),
                                                                         _bits(lam)[sel])


def test_octets_change_the_bits():
    """On a table whose blocks pass the octet test the octet variants do sum
    far blocks by octets: their bits differ from the pair twin's."""
    g = np.random.default_rng(8)
    nodes = inputs.equispaced(1001)
    vals = g.standard_normal(1001)
    pts = g.uniform(-1, 1, 30000)
    for vid, twin in TWIN.items():
        assert not torch.equal(_run(nodes, vals, 4, pts, vid)[0], _run(nodes, vals, 4, pts, twin)[0])


def test_small_workspace_and_failing_table_take_the_pair_twin():
    """Without room for the sorted points the call runs the pair twin; a
    table with a block that fails the octet test (one block twenty times
    wider than the spacing around it) runs the octet launch without octets:
    both give the twin's bits."""
    g = np.random.default_rng(9)
    nodes = inputs.equispaced(1001)
    vals = g.standard_normal(1001)
    pts = g.uniform(-1, 1, 30000)
    h = np.ones(1000)
    h[16 * 20:16 * 20 + 15] = 20.0
    wide = np.concatenate([[0.0], np.cumsum(h)])
    wide = -1.0 + 2.0 * wide / wide[-1]
    for vid, twin in TWIN.items():
        a = _run(nodes, vals, 5, pts, vid, ws_m=0)
        b = _run(nodes, vals, 5, pts, twin)
        assert all(np.array_equal(_bits(u), _bits(v)) for u, v in zip(a, b)), vid
        a = _run(wide, vals, 5, pts, vid)
        b = _run(wide, vals, 5, pts, twin)
        assert all(np.array_equal(_bits(u), _bits(v)) for u, v in zip(a, b)), vid


def _many(tables, pts, vid):
    """fh_eval_prepared_many over prepared (nodes, values, d) tables."""
    lib = fh.load()
    n, m, K = tables[0][0].size, len(pts), len(tables)
    ws_bytes = fh.workspace_size(fh.FH_OP_EVAL, n, m, max(t[2] for t in tables))
    wss = [fh.Workspace(DEV, ws_bytes) for _ in tables]
    s, P = fh._stream(torch.device(DEV)), fh._ptr
    keep = []
    for (nodes, vals, d), w in zip(tables, wss):
        xn, f = _t(nodes), _t(vals)
        keep += [xn, f]
        assert lib.fh_prepare(P(xn), P(f), n, d, None, fh.FH_FP64, ctypes.c_void_p(w.buf.data_ptr()),
                              ws_bytes, s) == 0
    x = _t(pts)
    r = torch.empty((K, m), dtype=torch.float64, device=DEV)
    lam = torch.empty_like(r)
    arr = lambda vs: (ctypes.c_void_p * K)(*vs)
    fh.tune_force("fp64", vid)
    try:
        st = lib.fh_eval_prepared_many(arr([w.buf.data_ptr() for w in wss]), ws_bytes, K, n,
                                       fh.FH_FP64, P(x), m, arr([r[i].data_ptr() for i in range(K)]),
                                       arr([lam[i].data_ptr() for i in range(K)]), s)
    finally:
        fh.tune_force("fp64", -1)
    torch.cuda.synchronize()
    assert st == 0
    return r, lam


def test_many_tables_each_with_the_bits_of_its_own_call():
    """One launch over several tables sorts the points by the first table's
    blocks; a table with other nodes is still served correctly (each block's
    choice uses the table's own nodes), and every table gets the bits of its
    own fh_eval_prepared call."""
    g = np.random.default_rng(10)
    n = 1001
    eq, ch = inputs.equispaced(n), inputs.cheb2(n)
    vals = g.standard_normal(n)
    tables = [(eq, vals, 3), (ch, vals, 2), (eq, np.cos(eq), 8)]
    pts = g.uniform(-1, 1, 40000)
    r, lam = _many(tables, pts, 25)
    for i, (nodes, v, d) in enumerate(tables):
        r1, lam1 = _run(nodes, v, d, pts, 25)
        assert np.array_equal(_bits(r[i]), _bits(r1)) and np.array_equal(_bits(lam[i]), _bits(lam1))


def test_log_reports_the_twin_for_a_small_workspace():
    """FH_LOG=1: a call whose workspace has no room for the sorted points
    says which pair variant runs instead of the octet variant."""
    import os
    import subprocess
    import sys
    code = (
        "import numpy as np, torch\n"
        "from paper_1606_06508_amd import fh, inputs\n"
        "x = torch.from_numpy(inputs.equispaced(1001)).cuda()\n"
        "p = torch.rand(5000, dtype=torch.float64, device='cuda') * 2 - 1\n"
        "nb = fh.workspace_size(fh.FH_OP_EVAL, 1001, 0, 3)\n"
        "ws = torch.zeros(nb, dtype=torch.uint8, device='cuda')\n"
        "r = torch.empty_like(p)\n"
        "fh.tune_force('fp64', 25)\n"
        "st = fh.load().fh_eval(fh._ptr(x), fh._ptr(x), 1001, 3, fh._ptr(p), 5000, fh._ptr(r),\n"
        "                       None, None, fh.FH_FP64, fh._ptr(ws), nb, fh._stream(x.device))\n"
        "torch.cuda.synchronize()\n"
        "print(st)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=root, env=dict(os.environ, FH_LOG="1"))
    assert p.returncode == 0 and p.stdout.strip() == "0", p.stderr
    assert "variant 25 has no workspace room for the sorted points" in p.stderr
    assert "variant 22 runs" in p.stderr
