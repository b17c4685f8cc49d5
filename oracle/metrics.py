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

The oracle's own accuracy bounds what any comparison can show: its
compensated D = sum a_k is good to about u |D| + n u^2 L (L = sum |a_k|), so
points whose Lambda = L/|D| approaches 1/(n u^2) have no correct digits on
either side; such shapes (d = n-1 on many equispaced nodes) are not used as
parity cases.
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


def parity(r, lam, r_o, lam_o, s_o):
    """Returns a dict of max errors (NaN-consistent points excluded from the
    maxima; NaN mismatches are counted separately)."""
    out = {}
    if r is not None:
        nan_o, nan_g = np.isnan(r_o), np.isnan(r)
        out["nan_mismatch_r"] = int(np.count_nonzero(nan_o != nan_g))
        ok = ~nan_o & ~nan_g
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
    if lam is not None:
        nan_o, nan_g = np.isnan(lam_o), np.isnan(lam)
        out["nan_mismatch_lam"] = int(np.count_nonzero(nan_o != nan_g))
        ok = ~nan_o & ~nan_g
        el = np.abs(lam[ok] - lam_o[ok]) / lam_o[ok]
        out["e_rel_lam_max"] = float(el.max()) if el.size else 0.0
        ec = el / (1.0 + lam_o[ok])
        out["e_cond_lam_max"] = float(ec.max()) if ec.size else 0.0
    return out


def check_split(stats, tol=SPLIT_TOL):
    """Asserts the FP32-split bar on a parity() dict."""
    assert stats["nan_mismatch_r"] == 0 and stats["nan_mismatch_lam"] == 0, stats
    assert stats["e_cond_max"] <= tol, stats
    assert stats["e_cond_lam_max"] <= tol, stats


def check_fp64(stats, tol=FP64_TOL, lam_metric="rel"):
    """Asserts the binary64 bar on a parity() dict (lam_metric "rel" for the
    workloads, "cond" for arbitrary shapes)."""
    if "e_cond_max" in stats:
        assert stats["nan_mismatch_r"] == 0, stats
        assert stats["e_cond_max"] <= tol, stats
        assert stats["e_rel_max_well_conditioned"] <= tol, stats
    if "e_rel_lam_max" in stats:
        assert stats["nan_mismatch_lam"] == 0, stats
        key = "e_rel_lam_max" if lam_metric == "rel" else "e_cond_lam_max"
        assert stats[key] <= tol, stats
