"""Parity metrics between a computed result and the FP64 oracle.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark's CPU leg).

Definitions (r_o, Lambda_o, S_o from the oracle; r, Lambda from the path):
  e_cond(r)   = |r - r_o| / S_o,  S_o = sum|a_k f_k|/|D| + |r_o| Lambda_o,
                the scale of the rounding error of any evaluation of the
                second form (plain relative error is unbounded near zeros
                of r, for every algorithm including the oracle);
  e_rel(r)    = |r - r_o| / |r_o|, reported unrestricted and checked where
                the condition number kappa = S_o / |r_o| is at most 100;
  e_rel(Lam)  = |Lambda - Lambda_o| / Lambda_o, the bar on the workloads
                (whose Lebesgue functions stay below a few hundred);
  e_cond(Lam) = |Lambda - Lambda_o| / (Lambda_o (1 + Lambda_o)), the bar on
                arbitrary shapes: D = sum a_k has condition number Lambda, so
                any binary64 evaluation of Lambda carries a relative error of
                order u (1 + Lambda) (e.g. d = n-1 on many equispaced nodes,
                where Lambda grows like 2^n).
Exact hits are compared bit-for-bit.

Conditioning limit.  Every term a_k = w_k / (x - x_k) carries a rounding
error of order u |a_k| in any evaluation (the oracle's included; its
compensation only removes the summation error), so a computed D is off by
up to c u L (L = sum |a_k|), a relative eta = c u Lambda.  The errors above
are first-order statements; to all orders, r^ - r = (dN / D - r dD / D) /
(1 + dD / D), so e_cond(r) and e_cond(Lambda) grow by at most 1 / (1 - eta)
and stay bounded while eta < 1.  FH interpolants on strongly non-uniform
nodes reach large Lambda (Chebyshev nodes: Lambda ~ 3e7 at n = 300, d = 6
and up to ~1e20 at n = 2048, d = 10).  Three bands, by the oracle's Lambda:
  Lambda <= lam_max (2^40, u Lambda <= 2^-13): the first-order bars;
  lam_max < Lambda <= lam_cap (2^48, u Lambda <= 2^-5): the same bars times
    k = Lambda / lam_max (the "Lambda-scaled" bar): 1 / (1 - c u Lambda) <= k
    holds for c <= 2^13 (k - 1) / k^2, i.e. for every c up to 31 over the
    whole band (k <= 256) and for larger c lower in it;
  Lambda > lam_cap: counted (n_beyond_lam_cap), not compared -- with
    c ~ 10..30, eta approaches 1 there and no evaluation has correct digits.
The FP32-split kernels recompute in binary64 every point whose binary32
terms give a Lebesgue function above 2^14 (their conditioning guard), so
the split bar applies on the same bands.
"""
import numpy as np

FP64_TOL = 1e-13          # binary64 path: every metric below
KAPPA_MAX = 100.0
# FP32-split path: e_cond(r) and e_cond(Lambda).  A binary32 tile sum of 32
# terms carries at most about 32 u32 relative to the sum of the terms'
# absolute values, plus a few u32 from the rounding of the difference, the
# reciprocal and the scaled weight: about 40 u32 = 2.4e-6; the stated bound
# leaves a factor of about three, 2^-17 (~134 u32).
SPLIT_TOL = 2.0 ** -17
FP64_LAMBDA_MAX = 2.0 ** 40
# the split value kernels send points beyond their guard (Lambda^ > 2^14) to
# binary64, so their bar covers the binary64 bands
SPLIT_LAMBDA_MAX = FP64_LAMBDA_MAX
LAMBDA_CAP = 2.0 ** 48
# first-order statement of the binary32 terms (error-statement tests) and
# the split derivative and adjoint kernels, which have no guard: points with
# Lambda up to 2^14 (about 40 u32 Lambda <= 0.04)
SPLIT_TERMS_LAMBDA_MAX = 2.0 ** 14
# Gradients (adjoint), measured against the sums of the absolute values of
# each component's terms (grad_scales): binary64 1e-12 (about 10^4 u, room
# for the plain chunked sums of the kernels against the oracle's compensated
# ones); FP32-split 2^-17, as for the values (binary32 tile sums of 32 terms).
GRAD_TOL = 1e-12
SPLIT_GRAD_TOL = 2.0 ** -17


def lambda_scale(lam):
    """Scale of the rounding error of Lambda = L / |D|: Lambda (1 + Lambda),
    the largest first-order change of Lambda per unit relative error when
    every term of L = sum |a_k| and of D = sum a_k carries an error of its
    own (d Lambda / d(L term k) = |b_k|, d Lambda / d(D term k) =
    -Lambda b_k)."""
    return lam * (1.0 + lam)


def parity(r, lam, r_o, lam_o, s_o, lam_max=FP64_LAMBDA_MAX, lam_cap=LAMBDA_CAP):
    """Returns a dict of max errors: the first-order bars over the points
    whose oracle Lambda is at most lam_max (all points when lam_o is None),
    the Lambda-scaled maxima (e_cond / (Lambda / lam_max)) over the points
    in (lam_max, lam_cap], and the counts of each band; NaN-consistent
    points are excluded from the maxima and NaN mismatches counted
    separately (over all points)."""
    out = {"lam_max": float(lam_max), "lam_cap": float(lam_cap)}
    shape = np.shape(r_o if r_o is not None else lam_o)
    keep = np.ones(shape, dtype=bool)
    mid = np.zeros(shape, dtype=bool)
    growth = np.ones(shape)
    if lam_o is not None:
        keep = ~(lam_o > lam_max)            # NaN Lambda is kept (NaN checks)
        mid = (lam_o > lam_max) & (lam_o <= lam_cap)
        growth = np.where(mid, lam_o / lam_max, 1.0)
        out["n_beyond_lam_max"] = int(np.count_nonzero(~keep))
        out["n_lambda_scaled"] = int(np.count_nonzero(mid))
        out["n_beyond_lam_cap"] = int(np.count_nonzero(lam_o > lam_cap))
    if r is not None:
        nan_o, nan_g = np.isnan(r_o), np.isnan(r)
        out["nan_mismatch_r"] = int(np.count_nonzero(nan_o != nan_g))
        ok = ~nan_o & ~nan_g & keep
        err = np.abs(r[ok] - r_o[ok])
        s = s_o[ok]
        with np.errstate(divide="ignore", invalid="ignore"):
            econd = np.where(s > 0, err / s, np.where(err == 0, 0.0, np.inf))
            erel = np.where(r_o[ok] != 0, err / np.abs(r_o[ok]), np.where(err == 0, 0.0, np.inf))
            kappa = np.where(r_o[ok] != 0, s / np.abs(r_o[ok]), np.inf)
        out["e_cond_max"] = float(econd.max()) if econd.size else 0.0
        out["e_rel_max"] = float(erel.max()) if erel.size else 0.0
        well = kappa <= KAPPA_MAX
        out["e_rel_max_well_conditioned"] = float(erel[well].max()) if np.any(well) else 0.0
        out["e_rel_p9999"] = float(np.quantile(erel, 0.9999)) if erel.size else 0.0
        okm = ~nan_o & ~nan_g & mid
        em = np.abs(r[okm] - r_o[okm])
        with np.errstate(divide="ignore", invalid="ignore"):
            ecm = np.where(s_o[okm] > 0, em / s_o[okm], np.where(em == 0, 0.0, np.inf))
        out["e_cond_scaled_max"] = float((ecm / growth[okm]).max()) if ecm.size else 0.0
    if lam is not None:
        nan_o, nan_g = np.isnan(lam_o), np.isnan(lam)
        out["nan_mismatch_lam"] = int(np.count_nonzero(nan_o != nan_g))
        ok = ~nan_o & ~nan_g & keep
        dl = np.abs(lam[ok] - lam_o[ok])
        el = dl / lam_o[ok]
        out["e_rel_lam_max"] = float(el.max()) if el.size else 0.0
        ec = dl / lambda_scale(lam_o[ok])
        out["e_cond_lam_max"] = float(ec.max()) if ec.size else 0.0
        okm = ~nan_o & ~nan_g & mid
        ecm = np.abs(lam[okm] - lam_o[okm]) / lambda_scale(lam_o[okm])
        out["e_cond_lam_scaled_max"] = float((ecm / growth[okm]).max()) if ecm.size else 0.0
    return out


def check_split(stats, tol=SPLIT_TOL):
    """Asserts the FP32-split bar on a parity() dict computed with
    lam_max <= SPLIT_LAMBDA_MAX: the first-order band and the Lambda-scaled
    band."""
    assert stats["lam_max"] <= SPLIT_LAMBDA_MAX, stats
    assert stats["nan_mismatch_r"] == 0 and stats["nan_mismatch_lam"] == 0, stats
    assert stats["e_cond_max"] <= tol, stats
    assert stats["e_cond_lam_max"] <= tol, stats
    assert stats.get("e_cond_scaled_max", 0.0) <= tol, stats
    assert stats.get("e_cond_lam_scaled_max", 0.0) <= tol, stats


def check_fp64(stats, tol=FP64_TOL, lam_metric="rel"):
    """Asserts the binary64 bar on a parity() dict (lam_metric "rel" for the
    workloads, "cond" for arbitrary shapes)."""
    if "e_cond_max" in stats:
        assert stats["nan_mismatch_r"] == 0, stats
        assert stats["e_cond_max"] <= tol, stats
        assert stats["e_rel_max_well_conditioned"] <= tol, stats
        assert stats.get("e_cond_scaled_max", 0.0) <= tol, stats
    if "e_rel_lam_max" in stats:
        assert stats["nan_mismatch_lam"] == 0, stats
        key = "e_rel_lam_max" if lam_metric == "rel" else "e_cond_lam_max"
        assert stats[key] <= tol, stats
        assert stats.get("e_cond_lam_scaled_max", 0.0) <= tol, stats


# ------------------------------------------------------------ gradients --
def weight_derivative_abs(x, d):
    """A[k, l] = sum over the terms of w_k of |d term / d x_l| (dense, small
    n): the scale of the chain dL/dx_l += sum_k dL/dw_k dw_k/dx_l."""
    n = x.size
    A = np.zeros((n, n))
    for k in range(n):
        for i in range(max(0, k - d), min(k, n - 1 - d) + 1):
            win = [j for j in range(i, i + d + 1) if j != k]
            T = 1.0 / np.prod([x[k] - x[j] for j in win]) if win else 1.0
            for l in win:
                A[k, l] += abs(T / (x[k] - x[l]))
            A[k, k] += abs(T) * sum(1.0 / abs(x[k] - x[j]) for j in win)
    return A


def grad_scales(nodes, vals, d, pts, g):
    """The adjoint's error scales (s_df[n], s_dx[m], s_dxd[n] for dL/dx_k at
    fixed weights, s_dw[n]) in numpy, by the definition of fho_grad_scales:
    each is the largest first-order change of its gradient component per
    unit relative error when every term an evaluation of the adjoint forms
    carries an error of its own -- the terms of N_p and D_p (which reach the
    gradients through r_p = N_p / D_p and c_p = g_p / D_p) and the terms of
    the node sums over points.  With b_k = a_pk / D_p, t_pk = 1/(x_p - x_k)
    and B_pk = |f_k| + |r_p| + Lambda_p |2 r_p - f_k| + sum_j |b_j f_j|:
      s_df[k] = sum_p |g_p b_k| (1 + Lambda_p),
      s_dw[k] = sum_p |g_p / D_p| |t_pk| B_pk,
      s_dxd[k] = sum_p |g_p b_k t_pk| B_pk,
      s_dx[p] = |g_p| S'(x_p), S' the derivative's scale (dL/dx_p = g_p r'):
        |e| sum|b_k f_k| + |r e + r'| Lambda + sum|b_k t_k| (|r| + |f_k|),
        e = sum_k b_k t_k.
    Exact hits x_p == x_j contribute |g_p| to s_df[j] and |g_p| times the
    sum of |terms| of the node formula to s_dx[p] and s_dxd[j]."""
    from . import oracle
    w = oracle.weights(nodes, d)
    ok = np.isfinite(pts) & ~np.isin(pts, nodes)
    s_df = np.zeros(nodes.size)
    s_dw = np.zeros(nodes.size)
    s_dxd = np.zeros(nodes.size)
    s_dx = np.zeros(pts.size)
    af_abs = np.abs(vals)
    idx = np.flatnonzero(ok)
    for lo in range(0, idx.size, 2000):
        sel = idx[lo:lo + 2000]
        T = 1.0 / (pts[sel, None] - nodes[None, :])
        a = w[None, :] * T
        af = a * vals[None, :]
        D = a.sum(1)
        r = af.sum(1) / D
        lam = np.abs(a).sum(1) / np.abs(D)
        sbf = np.abs(af).sum(1) / np.abs(D)
        e = (a * T).sum(1) / D
        dr = (r * (a * T).sum(1) - (af * T).sum(1)) / D
        b = np.abs(a) / np.abs(D)[:, None]
        s_dx[sel] = np.abs(g[sel]) * (
            np.abs(e) * sbf + np.abs(r * e + dr) * lam
            + (b * np.abs(T) * (np.abs(r)[:, None] + af_abs[None, :])).sum(1))
        B = (af_abs[None, :] + np.abs(r)[:, None]
             + lam[:, None] * np.abs(2.0 * r[:, None] - vals[None, :]) + sbf[:, None])
        gb = np.abs(g[sel])[:, None] * b
        s_df += (gb * (1.0 + lam)[:, None]).sum(0)
        s_dw += (np.abs(g[sel] / D)[:, None] * np.abs(T) * B).sum(0)
        s_dxd += (gb * np.abs(T) * B).sum(0)
    for p in np.flatnonzero(np.isin(pts, nodes)):
        j = int(np.searchsorted(nodes, pts[p]))
        others = np.arange(nodes.size) != j
        rp_abs = np.sum(np.abs(w[others] / w[j]) * np.abs(vals[others] - vals[j])
                        / np.abs(nodes[j] - nodes[others]))
        s_df[j] += abs(g[p])
        s_dx[p] = abs(g[p]) * rp_abs
        s_dxd[j] += abs(g[p]) * rp_abs
    return s_df, s_dx, s_dxd, s_dw


def grad_errors(gv, gx, gn, o, scales, nodes=None, d=None):
    """Max of |path - oracle| / scale per gradient (the node gradient only
    when nodes and d are given: its scale adds the dense weight chain).
    NaN patterns of dL/dx must agree (counted in nan_mismatch_dx)."""
    s_df, s_dx, s_dxd, s_dw = scales
    tiny = 1e-300
    out = {}
    if gv is not None:
        out["dvalues"] = float(np.max(np.abs(gv - o["d_values"]) / (s_df + tiny)))
    if gx is not None:
        fin = np.isfinite(o["d_points"])
        out["nan_mismatch_dx"] = int(np.count_nonzero(np.isfinite(gx) != fin))
        out["dpoints"] = float(np.max(np.abs(gx[fin] - o["d_points"][fin]) / (s_dx[fin] + tiny))
                               if np.any(fin) else 0.0)
    if gn is not None and nodes is not None:
        s_dn = s_dxd + weight_derivative_abs(nodes, d).T @ s_dw
        out["dnodes"] = float(np.max(np.abs(gn - o["d_nodes"]) / (s_dn + tiny)))
    return out


def check_grad(errors, tol=GRAD_TOL):
    """Asserts a grad_errors() dict against tol."""
    assert errors.get("nan_mismatch_dx", 0) == 0, errors
    for k in ("dvalues", "dpoints", "dnodes"):
        if k in errors:
            assert errors[k] <= tol, errors
