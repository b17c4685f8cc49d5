"""fh_eval_noalloc, the entry point that allocates nothing (its node table
sits in a fixed device array of the library): called through the C ABI, it
returns the bits of fh_eval on the same problem, call after call on the one
shared array -- a large problem, then a smaller one, so stale table entries
beyond the second table would show -- in binary64 and FP32-split, with and
without Lambda; and the oracle's bar holds."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _problem(n, m, seed):
    g = np.random.default_rng(seed)
    nodes = inputs.jittered_nodes(n, g)
    om, amp = inputs.sines_params(g)
    vals = inputs.sines(nodes, om, amp)
    pts = g.uniform(-1.0, 1.0, m)
    pts[: min(m, 7)] = nodes[g.choice(n, min(m, 7), replace=False)]  # exact hits
    return nodes, vals, pts


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("lebesgue", [True, False])
def test_noalloc_equals_fh_eval_on_consecutive_calls(precision, lebesgue):
    # the largest table the array holds, then a smaller one (ragged sizes)
    shapes = [(fh.FH_NOALLOC_MAX_NODES, 20_011, 5, 11), (301, 4_099, 3, 12)]
    for n, m, d, seed in shapes:
        nodes, vals, pts = _problem(n, m, seed)
        xn, f, x = _t(nodes), _t(vals), _t(pts)
        r = torch.full((m,), np.nan, dtype=torch.float64, device=DEV)
        lam = torch.full((m,), np.nan, dtype=torch.float64, device=DEV) if lebesgue else None
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(DEV)
        fh.evaluate_noalloc(xn, f, d, x, r, lambda_out=lam, precision=precision)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(DEV) == before
        ref = fh.evaluate(xn, f, d, x, lebesgue=lebesgue, precision=precision)
        r_ref, lam_ref = ref if lebesgue else (ref, None)
        torch.cuda.synchronize()
        assert torch.equal(r, r_ref), (precision, n, m)
        if lebesgue:
            assert torch.equal(lam, lam_ref), (precision, n, m)
        # the oracle's bar on a sample of the points (and every hit)
        sel = np.unique(np.concatenate([np.arange(7), np.random.default_rng(seed).choice(
            m, 1500, replace=False)]))
        r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, pts[sel])
        idx = torch.from_numpy(sel).to(DEV)
        st = metrics.parity(r[idx].cpu().numpy(), lam[idx].cpu().numpy() if lebesgue else None,
                            r_o, lam_o, s_o,
                            metrics.FP64_LAMBDA_MAX if precision == "fp64" else
                            metrics.SPLIT_LAMBDA_MAX)
        if precision == "fp64":
            metrics.check_fp64(st)
        else:
            assert st["nan_mismatch_r"] == 0 and st["e_cond_max"] <= metrics.SPLIT_TOL, st
        assert np.array_equal(r[:7].cpu().numpy(), r_o[:7])


def test_noalloc_refuses_a_table_beyond_its_array():
    nodes, vals, pts = _problem(fh.FH_NOALLOC_MAX_NODES + 1, 64, 13)
    r = torch.empty(64, dtype=torch.float64, device=DEV)
    with pytest.raises(fh.FhError) as e:
        fh.evaluate_noalloc(_t(nodes), _t(vals), 3, _t(pts), r)
    assert e.value.code == fh.FH_E_TOO_LARGE


def test_noalloc_valid_call_after_invalid_nodes():
    """Each call clears the array's status block and repacks the table: a
    call with valid nodes after one with repeated nodes (whose outputs are
    unspecified) returns the bits of fh_eval."""
    nodes, vals, pts = _problem(257, 3000, 14)
    bad = nodes.copy()
    bad[10] = bad[9]
    r = torch.empty(3000, dtype=torch.float64, device=DEV)
    fh.evaluate_noalloc(_t(bad), _t(vals), 2, _t(pts), r)
    fh.evaluate_noalloc(_t(nodes), _t(vals), 2, _t(pts), r)
    ref = fh.evaluate(_t(nodes), _t(vals), 2, _t(pts))
    torch.cuda.synchronize()
    assert torch.equal(r, ref)
