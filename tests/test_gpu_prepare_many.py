"""fh_prepare_many: the tables of several degrees packed in one launch are
the tables fh_prepare writes, so every evaluation from them equals fh_eval
bit for bit (r and Lambda, hits and NaN/inf points included)."""
import numpy as np
import pytest
import torch

from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _bits_equal(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
        a[~np.isnan(a)].view(np.uint64), b[~np.isnan(b)].view(np.uint64))


@pytest.mark.parametrize("n,degrees", [(1001, range(9)), (257, [3, 0, 7, 7, 2]), (1, [0]),
                                       (40, [0, 39, 5])])
def test_tables_equal_single_prepare(n, degrees):
    g = np.random.default_rng(n)
    c = inputs.sines_workload(n=n, m=20000) if n > 1 else None
    nodes = c["nodes"] if c else np.array([0.25])
    vals = c["values"] if c else np.array([1.5])
    pts = np.concatenate([g.uniform(-1, 1, 20000), nodes[::5], [np.nan, np.inf, -np.inf]])
    tn, tv, tx = (torch.from_numpy(a).to(DEV) for a in (nodes, vals, pts))
    preps = fh.prepare_many(tn, tv, degrees)
    for d, p in zip(degrees, preps):
        r, lam = p(tx, lebesgue=True)
        r1, lam1 = fh.evaluate(tn, tv, d, tx, lebesgue=True)
        torch.cuda.synchronize()
        assert _bits_equal(r, r1) and _bits_equal(lam, lam1), d
        assert p.ws.status() == (fh.FH_OK, 0)


def test_lebesgue_only_tables():
    c = inputs.sines_workload(n=301, m=5000)
    tn, tx = torch.from_numpy(c["nodes"]).to(DEV), torch.from_numpy(c["points"]).to(DEV)
    preps = fh.prepare_many(tn, None, [1, 4])
    for d, p in zip([1, 4], preps):
        lam = p(tx, want_r=False, lebesgue=True)
        lam1 = fh.lebesgue(tn, d, tx)
        torch.cuda.synchronize()
        assert _bits_equal(lam, lam1), d
