"""Pins of the error scales that every parity bar divides by.

S (values), Lambda (1 + Lambda) (the Lebesgue function), S' (derivative)
and the adjoint's scales (dL/df_k, dL/dx_p, dL/dw_k, dL/dx_k) are each
defined as the largest first-order change of the result per unit relative
error in the terms the computation forms.  They are checked here against
an exact perturbation experiment (no formula for the scale) and against
the same quantity assembled from the exact blend-form cardinals, for the C
oracle and for the numpy scales the GPU tests use (scale_pins.py).  A
deliberately inflated or truncated scale in a copy of the oracle fails
these checks (test_oracle_scale_mutants.py).
"""
import numpy as np
import pytest

import scale_pins
from oracle import metrics, oracle
from paper_1606_06508_amd import inputs


def _case(n, d, seed, jitter=0.3, hits=(1,)):
    rng = np.random.default_rng(seed)
    x = inputs.equispaced(n)
    if n > 2:
        x[1:-1] += rng.uniform(-jitter, jitter, n - 2) * (2.0 / (n - 1))
    f = rng.standard_normal(n)
    pts = np.concatenate([rng.uniform(-1.0, 1.0, 4), [1.3, -1.1],
                          x[[h for h in hits if h < n]], [x[0] + 1e-9]])
    g = rng.standard_normal(pts.size)
    return x, f, pts, g


CASES = [(2, 1, 1), (4, 0, 2), (5, 2, 3), (7, 3, 4), (8, 7, 5), (9, 4, 6)]


@pytest.mark.parametrize("n,d,seed", CASES)
def test_value_scale(n, d, seed):
    x, f, pts, _ = _case(n, d, seed)
    scale_pins.check_value_scale(oracle, x, f, d, pts)


@pytest.mark.parametrize("n,d,seed", CASES)
def test_lambda_scale(n, d, seed):
    x, _, pts, _ = _case(n, d, seed)
    scale_pins.check_lambda_scale(metrics.lambda_scale, x, oracle.weights(x, d), d, pts)


@pytest.mark.parametrize("n,d,seed", CASES)
def test_derivative_scale(n, d, seed):
    x, f, pts, _ = _case(n, d, seed)
    scale_pins.check_deriv_scale(oracle, x, f, d, pts)


@pytest.mark.parametrize("n,d,seed", [(3, 1, 11), (5, 2, 12), (6, 3, 13), (7, 6, 14)])
def test_adjoint_scales_c(n, d, seed):
    x, f, pts, g = _case(n, d, seed, hits=(2,))
    pts = pts[:5]  # keep the exact adjoint experiment small
    pts = np.concatenate([pts, [x[2], np.nan]])
    g = np.resize(g, pts.size)
    scale_pins.check_grad_scales(oracle.grad_scales(x, f, d, pts, g, parts=True), oracle, x, f, d,
                                 pts, g)


@pytest.mark.parametrize("n,d,seed", [(3, 1, 21), (5, 2, 22), (6, 3, 23)])
def test_adjoint_scales_numpy(n, d, seed):
    x, f, pts, g = _case(n, d, seed)
    pts = np.concatenate([pts[:5], [x[1], np.nan]])
    g = np.resize(g, pts.size)
    s_df, s_dx, s_dxd, s_dw = metrics.grad_scales(x, f, d, pts, g)
    s_dn = s_dxd + metrics.weight_derivative_abs(x, d).T @ s_dw
    scale_pins.check_grad_scales((s_df, s_dx, s_dn, s_dw, s_dxd), oracle, x, f, d, pts, g)


def test_weight_chain_matrix_numpy():
    """metrics.weight_derivative_abs (the numpy scales' weight chain) equals
    exact central differences of the weight terms."""
    for n, d in ((4, 1), (7, 3), (6, 5)):
        x = inputs.equispaced(n) + np.random.default_rng(n).uniform(-0.2, 0.2, n) * (2.0 / (n - 1))
        A = scale_pins.weight_chain_abs(x, d)
        B = metrics.weight_derivative_abs(x, d)
        assert np.allclose(A, B, rtol=16 * (d + 2) * 2.0 ** -53, atol=0.0)
