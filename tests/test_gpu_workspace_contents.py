"""Every call writes each workspace byte it reads, apart from the status
block: results are bit for bit the same from a workspace whose bytes past
the first 256 are zero and from one filled with 0xFF (every binary64 there a
NaN).  The Workspace helper zero-fills only the status block."""
import numpy as np
import pytest
import torch

from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _pair(nbytes):
    """(zeroed, 0xFF-filled) workspaces with zero status blocks."""
    a, b = fh.Workspace(DEV, nbytes), fh.Workspace(DEV, nbytes)
    a.buf.zero_()
    b.buf.fill_(0xFF)
    b.buf[:256].zero_()
    return a, b


def _same(u, v):
    if u is None or v is None:
        assert u is None and v is None
        return
    assert torch.equal(torch.isnan(u), torch.isnan(v))
    assert torch.equal(u.nan_to_num(0.0), v.nan_to_num(0.0))


def _case(n=517, m=7001, d=4, seed=2):
    g = np.random.default_rng(seed)
    nodes = np.sort(inputs.equispaced(n) + g.uniform(-0.3, 0.3, n) / n)
    vals = g.standard_normal(n)
    pts = np.concatenate([g.uniform(-1.05, 1.05, m - 4), nodes[[0, 7, n - 1]], [np.nan]])
    return _t(nodes), _t(vals), d, _t(pts), _t(g.standard_normal(m))


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_eval_and_lebesgue(precision):
    nodes, vals, d, x, _ = _case()
    size = fh.workspace_size(fh.FH_OP_EVAL, nodes.numel(), x.numel(), d, precision)
    a, b = _pair(size)
    for ws in (a, b):
        ws.out = fh.evaluate(nodes, vals, d, x, lebesgue=True, precision=precision, ws=ws)
        ws.lam = fh.lebesgue(nodes, d, x, precision=precision, ws=ws)
        ws.der = fh.eval_deriv(nodes, vals, d, x, precision=precision, ws=ws)
    for u, v in zip(a.out + (a.lam,) + a.der, b.out + (b.lam,) + b.der):
        _same(u, v)


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_adjoints(precision):
    nodes, vals, d, x, g = _case()
    n, m = nodes.numel(), x.numel()
    a, b = _pair(fh.workspace_size(fh.FH_OP_BACKWARD, n, m, d, precision))
    ra = fh.eval_backward(nodes, vals, d, x, g, precision=precision, ws=a)
    rb = fh.eval_backward(nodes, vals, d, x, g, precision=precision, ws=b)
    for u, v in zip(ra, rb):
        _same(u, v)
    for derivative in (False, True):
        a, b = _pair(fh.workspace_size(fh.FH_OP_BACKWARD_SAVED, n, m, d, precision))
        outs = []
        for ws in (a, b):
            r, st = fh.eval_forward(nodes, vals, d, x, precision=precision, ws=ws,
                                    derivative=derivative)
            outs.append((r,) + fh.eval_backward_saved(st, g))
        for u, v in zip(*outs):
            _same(u, v)


def test_lebesgue_max_and_multi():
    nodes, vals, d, x, _ = _case(n=301, m=3001)
    n = nodes.numel()
    a, b = _pair(fh.workspace_size(fh.FH_OP_LEBESGUE_MAX, n, 0, d))
    la = fh.lebesgue_max(nodes, d, ws=a)
    lb = fh.lebesgue_max(nodes, d, ws=b)
    for u, v in zip(la, lb):
        _same(u, v)
    a, b = _pair(fh.multi_workspace_size(n, 5))
    vals5 = vals.repeat(5, 1).contiguous()
    ma = fh.eval_multi(nodes, vals5, [0, 1, 2, 3, 4], x, lebesgue=True, ws=a)
    mb = fh.eval_multi(nodes, vals5, [0, 1, 2, 3, 4], x, lebesgue=True, ws=b)
    for u, v in zip(ma, mb):
        _same(u, v)
