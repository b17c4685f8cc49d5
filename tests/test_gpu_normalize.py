"""Parity of the HIP normalization kernels (include/nrm.h) with the
normalization oracle: bit for bit, since both run the same IEEE operations
in the same order (NaN positions must agree; NaN payloads are not
compared).  Inputs span the whole exponent range of each format, with zero,
NaN, infinite, subnormal and near-overflow vectors; the full 10^8-vector
workloads are checked bit for bit at every vector and through properties
that hold for every vector."""
import numpy as np
import pytest
import torch

from oracle import nrm
from paper_1606_06508_amd import inputs
from paper_1606_06508_amd.normalize import normalize

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
DTYPES = {"f32": np.float32, "f64": np.float64}
METHODS = ["scaling", "quotient", "quotient_pivot", "naive"]


def _special(dim, dt):
    fi = np.finfo(dt)
    tiny = float(fi.smallest_subnormal)
    rows = [[0.0] * dim, [-0.0] * dim, [tiny] * dim, [float(fi.max)] * dim,
            [float(fi.max)] + [tiny] * (dim - 1), [1.0] + [0.0] * (dim - 1),
            [0.0] * (dim - 1) + [-tiny], [np.inf] + [1.0] * (dim - 1),
            [3.0, 4.0, 12.0, 84.0][:dim], [-2.0 ** -1000, 2.0 ** -1010, 0.0, 1e-320][:dim],
            [1.0] * (dim - 1) + [-np.inf], [np.nan] + [0.0] * (dim - 1)]
    for k in range(dim):  # NaN in every position next to zeros (the zero exits)
        v = [0.0] * dim
        v[k] = np.nan
        rows.append(v)
    return np.array(rows, dtype=np.float64).astype(dt)


def _cases(dim, dt, n=20011, salt=0):
    x = [inputs.nrm_vectors(n, dim, dt, salt=salt), _special(dim, dt)]
    if dim == 4:
        x.append(inputs.near_unit_quaternions(2000, dt, salt=salt))
    return np.ascontiguousarray(np.concatenate(x))


def _same(a, b):
    """Bit equality with NaN positions (not payloads) compared."""
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb)
    assert np.array_equal(a[~na].view(np.uint8), b[~nb].view(np.uint8))


@pytest.mark.parametrize("sfx", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3, 4])
@pytest.mark.parametrize("method", METHODS)
def test_bitwise_against_oracle(method, dim, sfx):
    if method == "quotient_pivot" and dim != 3:
        pytest.skip("Algorithm 2 is three dimensional")
    dt = DTYPES[sfx]
    x = _cases(dim, dt, salt=dim)
    r_o, xh_o = nrm.normalize(x, method)
    xt = torch.from_numpy(x).to(DEV)
    r, xh = normalize(xt, method=method)
    torch.cuda.synchronize()
    _same(r.cpu().numpy(), r_o)
    _same(xh.cpu().numpy(), xh_o)
    # struct-of-arrays layout: the same bits
    r2, xh2 = normalize(xt.t().contiguous(), method=method, layout="soa")
    torch.cuda.synchronize()
    _same(r2.cpu().numpy(), r_o)
    _same(xh2.t().cpu().numpy(), xh_o)


@pytest.mark.parametrize("sfx", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3, 4])
def test_full_workload_every_row_and_properties(dim, sfx):
    """10^8 vectors drawn on the device (the benchmark's workload): every
    vector against the oracle bit for bit (row slices of 10^7 copied to the
    host; no index tensors), and for every vector: finite input -> finite
    direction of norm 1 within a few u, NaN input <-> NaN output, zero input
    <-> r = 0."""
    dt = DTYPES[sfx]
    n = 10 ** 8
    x = inputs.nrm_vectors_device(n, dim, sfx, DEV)
    r, xh = normalize(x)
    torch.cuda.synchronize()
    for lo in range(0, n, 10 ** 7):
        hi = min(n, lo + 10 ** 7)
        r_o, xh_o = nrm.normalize(x[lo:hi].cpu().numpy(), "scaling")
        _same(r[lo:hi].cpu().numpy(), r_o)
        _same(xh[lo:hi].cpu().numpy(), xh_o)
        del r_o, xh_o
    # whole-tensor masked reductions
    nan_in = torch.isnan(x).any(dim=1)
    assert (torch.isfinite(x) | nan_in[:, None]).all()  # the recipe draws no infinities
    assert torch.equal(torch.isnan(r), nan_in)
    assert torch.equal(torch.isnan(xh).any(dim=1), nan_in)
    assert torch.equal(torch.isnan(xh).all(dim=1), nan_in)
    zero = (x == 0).all(dim=1)
    assert torch.equal((r == 0) & ~nan_in, zero & ~nan_in)
    nz = ~nan_in & ~zero
    assert (torch.isfinite(xh) | ~nz[:, None]).all()
    norm = torch.sqrt((xh.double() ** 2).sum(dim=1))
    dev = torch.where(nz, (norm - 1).abs(), torch.zeros_like(norm))
    u = 2.0 ** -24 if sfx == "f32" else 2.0 ** -53
    assert float(dev.max()) <= 8 * u
    del x, r, xh, norm, dev


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 4097])
def test_ragged_sizes_and_partial_outputs(n):
    x = _cases(3, np.float64, n=n, salt=n)[:n]
    r_o, xh_o = nrm.normalize(x, "scaling")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    r, xh = normalize(xt)
    r_only, none = normalize(xt, directions=False)
    none2, xh_only = normalize(xt, lengths=False)
    torch.cuda.synchronize()
    assert none is None and none2 is None
    for a in (r, r_only):
        _same(a.cpu().numpy(), r_o)
    for a in (xh, xh_only):
        _same(a.cpu().numpy(), xh_o)


def test_empty_input():
    x = torch.empty((0, 4), dtype=torch.float32, device=DEV)
    r, xh = normalize(x)
    assert r.numel() == 0 and xh.numel() == 0


def test_output_tensors_are_checked():
    """Caller-provided outputs of the wrong shape, dtype or layout are refused
    before any launch (a shorter r_out would otherwise be written past its
    end)."""
    x = torch.ones((100, 3), dtype=torch.float64, device=DEV)
    for bad in (dict(r_out=torch.empty(99, dtype=torch.float64, device=DEV)),
                dict(r_out=torch.empty(100, dtype=torch.float32, device=DEV)),
                dict(dir_out=torch.empty((100, 4), dtype=torch.float64, device=DEV)),
                dict(dir_out=torch.empty((3, 100), dtype=torch.float64, device=DEV).t())):
        with pytest.raises(ValueError):
            normalize(x, **bad)
