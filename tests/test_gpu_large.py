"""Arrays past 2^31 bytes: 3 * 10^8 points (2.4 GB per binary64 array), so
point indices times eight overflow 32 bits.  Outputs are checked against the
oracle on sampled points that include the first and the last ones, and the
non-finite count must be zero (every point is finite and inside the nodes).
Vector normalization gets 3 * 10^8 three-dimensional binary64 vectors
(7.2 GB in)."""
import numpy as np
import pytest
import torch

from oracle import metrics, nrm, oracle
from paper_1606_06508_amd import fh, inputs
from paper_1606_06508_amd.normalize import normalize

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
M = 300_000_000


def _points():
    g = torch.Generator(device=DEV)
    g.manual_seed(1606)
    return torch.rand(M, dtype=torch.float64, device=DEV, generator=g) * 2.0 - 1.0


def _sample():
    g = np.random.default_rng(5)
    return np.unique(np.concatenate([[0, 1, M - 2, M - 1], g.integers(0, M, 4000)]))


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_three_hundred_million_points(precision):
    nodes = inputs.equispaced(33)
    vals = np.cos(3 * nodes)
    x = _points()
    r, lam = fh.evaluate(torch.from_numpy(nodes).to(DEV), torch.from_numpy(vals).to(DEV), 3, x,
                         lebesgue=True, precision=precision)
    torch.cuda.synchronize()
    assert int((~torch.isfinite(r)).sum()) == 0 and int((~torch.isfinite(lam)).sum()) == 0
    idx = _sample()
    it = torch.from_numpy(idx).to(DEV)
    pts = x[it].cpu().numpy()
    r_o, lam_o, s_o = oracle.evaluate(nodes, vals, 3, pts)
    st = metrics.parity(r[it].cpu().numpy(), lam[it].cpu().numpy(), r_o, lam_o, s_o,
                        metrics.FP64_LAMBDA_MAX if precision == "fp64" else metrics.SPLIT_LAMBDA_MAX)
    if precision == "fp64":
        metrics.check_fp64(st)
    else:
        metrics.check_split(st)
    del x, r, lam
    torch.cuda.empty_cache()


def test_three_hundred_million_points_derivative():
    nodes = inputs.equispaced(33)
    vals = np.cos(3 * nodes)
    x = _points()
    _, dr = fh.eval_deriv(torch.from_numpy(nodes).to(DEV), torch.from_numpy(vals).to(DEV), 3, x,
                          want_r=False)
    torch.cuda.synchronize()
    idx = _sample()
    it = torch.from_numpy(idx).to(DEV)
    _, dr_o, s_o = oracle.eval_deriv(nodes, vals, 3, x[it].cpu().numpy())
    err = np.abs(dr[it].cpu().numpy() - dr_o) / s_o
    assert err.max() <= 1e-12
    del x, dr
    torch.cuda.empty_cache()


def test_three_hundred_million_vectors():
    n = M
    x = inputs.nrm_vectors_device(n, 3, "f64", DEV)
    r, xh = normalize(x)
    torch.cuda.synchronize()
    idx = torch.from_numpy(_sample()).to(DEV)
    r_o, xh_o = nrm.normalize(x[idx].cpu().numpy(), "scaling")
    for a, b in ((r[idx].cpu().numpy(), r_o), (xh[idx].cpu().numpy(), xh_o)):
        na, nb = np.isnan(a), np.isnan(b)
        assert np.array_equal(na, nb)
        assert np.array_equal(a[~na].view(np.uint64), b[~nb].view(np.uint64))
    del x, r, xh
    torch.cuda.empty_cache()
