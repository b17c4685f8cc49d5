"""Checks that pin the oracle's error scales to routes that share nothing
with its closed-form sums (used by test_oracle_scales.py on the oracle and
by test_oracle_scale_mutants.py on deliberately wrong copies of it).

Every scale is a worst-case first-order sensitivity: the largest change of
a result per unit relative error when every term the computation forms
carries a relative error of its own.  Two routes:

  perturbation  the computation is repeated in exact rational arithmetic
                with one term at a time perturbed by a relative 2^-100, and
                the changes of the result are added in absolute value
                (exact.term_sensitivities); no formula for the scale enters;
  cardinals     the scale assembled from the exact cardinal functions b_k of
                the blend form (a different algorithm from the second form
                the oracle sums) and exact central differences.

Each check raises AssertionError on a mismatch.
"""
from fractions import Fraction

import numpy as np

from oracle import exact

U = 2.0 ** -53
H = Fraction(1, 10 ** 30)


def _fr(v):
    return [Fraction(float(t)) for t in v]


def _rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def _non_hit_points(x, pts):
    return [float(t) for t in pts if np.isfinite(t) and not np.any(x == t)]


# ------------------------------------------------------------------ r, S --
def value_scale_routes(x, f, w, d, t):
    """(S by perturbation, S by cardinals, Lambda) at a non-hit point t."""
    xf, ff, wf = _fr(x), _fr(f), _fr(w)
    tf = Fraction(t)
    a = [wk / (tf - xk) for wk, xk in zip(wf, xf)]
    s_pert = exact.term_sensitivities(lambda g: sum(g[0]) / sum(g[1]),
                                      [[ak * fk for ak, fk in zip(a, ff)], a])
    b = exact.blend_cardinals(x, d, tf)
    r = sum(bk * fk for bk, fk in zip(b, ff))
    s_card = sum(abs(bk) * (abs(fk) + abs(r)) for bk, fk in zip(b, ff))
    lam = sum(abs(bk) for bk in b)
    return s_pert, s_card, float(lam)


def check_value_scale(orc, x, f, d, pts):
    """The oracle's S (fho_eval) equals both routes within 64 u (1 + Lambda)
    (its own rounding; D has condition number Lambda)."""
    _, _, s_o = orc.evaluate(x, f, d, pts)
    w = orc.weights(x, d)
    for t in _non_hit_points(x, pts):
        i = int(np.flatnonzero(pts == t)[0])
        s_pert, s_card, lam = value_scale_routes(x, f, w, d, t)
        tol = 64 * U * (1 + lam)
        assert _rel(s_o[i], s_pert) <= tol, ("S vs perturbation", t, s_o[i], float(s_pert))
        assert _rel(s_o[i], s_card) <= tol, ("S vs cardinals", t, s_o[i], float(s_card))


def check_lambda_scale(scale_fn, x, w, d, pts):
    """scale_fn(Lambda) (the Lambda bar's denominator) equals the
    perturbation sensitivity of Lambda = sum|a_k| / |sum a_k|."""
    xf, wf = _fr(x), _fr(w)
    for t in _non_hit_points(x, pts):
        tf = Fraction(t)
        a = [wk / (tf - xk) for wk, xk in zip(wf, xf)]
        s_pert = exact.term_sensitivities(lambda g: sum(g[0]) / abs(sum(g[1])),
                                          [[abs(ak) for ak in a], a])
        lam = float(sum(abs(ak) for ak in a) / abs(sum(a)))
        assert _rel(scale_fn(lam), s_pert) <= 64 * U * (1 + lam), ("Lambda scale", t)


# ----------------------------------------------------------------- r', S' --
def deriv_scale_routes(x, f, w, d, t):
    """(S' by perturbation of the four sums N, D, E, F, S' by cardinals,
    Lambda) at a non-hit point t."""
    xf, ff, wf = _fr(x), _fr(f), _fr(w)
    tf = Fraction(t)
    q = [1 / (tf - xk) for xk in xf]
    a = [wk * qk for wk, qk in zip(wf, q)]
    groups = [[ak * fk for ak, fk in zip(a, ff)], a, [ak * qk for ak, qk in zip(a, q)],
              [ak * fk * qk for ak, fk, qk in zip(a, ff, q)]]

    def rprime(g):
        N, D, E, Fs = (sum(v) for v in g)
        return (N / D * E - Fs) / D

    s_pert = exact.term_sensitivities(rprime, groups)
    b = exact.blend_cardinals(x, d, tf)
    bp = exact.cardinal_derivatives(x, d, tf, H)
    r = sum(bk * fk for bk, fk in zip(b, ff))
    rp = sum(bk * fk for bk, fk in zip(bp, ff))
    lam = sum(abs(bk) for bk in b)
    e = sum(bk * qk for bk, qk in zip(b, q))
    s_card = (abs(e) * sum(abs(bk * fk) for bk, fk in zip(b, ff)) + abs(r * e + rp) * lam
              + sum(abs(bk * qk) * (abs(r) + abs(fk)) for bk, qk, fk in zip(b, q, ff)))
    return s_pert, s_card, float(lam)


def node_deriv_scale(x, f, d, j):
    """S' at the node x_j: sum_k |b_k'(x_j)| |f_k - f_j| with the cardinal
    derivatives by exact central differences of the blend form."""
    ff = _fr(f)
    bp = exact.cardinal_derivatives(x, d, Fraction(float(x[j])), H)
    return sum(abs(bk) * abs(fk - ff[j]) for k, (bk, fk) in enumerate(zip(bp, ff)) if k != j)


def check_deriv_scale(orc, x, f, d, pts):
    """The oracle's S' (fho_eval_deriv) equals both routes within
    64 u (1 + Lambda)^2 off the nodes (its terms are products of sums that
    each carry D's conditioning), and the cardinal route at hits within
    16 n u."""
    _, _, sd_o = orc.eval_deriv(x, f, d, pts)
    w = orc.weights(x, d)
    for i, t in enumerate(pts):
        if not np.isfinite(t):
            continue
        hit = np.flatnonzero(x == t)
        if hit.size:
            ref = node_deriv_scale(x, f, d, int(hit[0]))
            assert _rel(sd_o[i], ref) <= 16 * x.size * U, ("S' at a node", t, sd_o[i], float(ref))
            continue
        s_pert, s_card, lam = deriv_scale_routes(x, f, w, d, float(t))
        tol = 64 * U * (1 + lam) ** 2
        assert _rel(sd_o[i], s_pert) <= tol, ("S' vs perturbation", t, sd_o[i], float(s_pert))
        assert _rel(sd_o[i], s_card) <= tol, ("S' vs cardinals", t, sd_o[i], float(s_card))


# -------------------------------------------------------------- adjoint --
def adjoint_scale_routes(x, f, w, d, pts, g):
    """Exact (s_df, s_dw, s_dxd) over the non-hit finite points by the
    perturbation route and by the cardinal route, as float arrays.

    The computation perturbed: per point N_p = sum_k a_pk f_k, D_p = sum_k
    a_pk, r_p = N_p / D_p, c_p = g_p / D_p; per node dL/df_k = sum_p c_p a_pk,
    dL/dw_k = sum_p (c_p f_k t_pk - c_p r_p t_pk), dL/dx_k (fixed weights) =
    sum_p (c_p a_pk f_k t_pk - c_p a_pk r_p t_pk); every term of every sum
    perturbed alone."""
    xf, ff, wf = _fr(x), _fr(f), _fr(w)
    n = len(xf)
    P = _non_hit_points(x, pts)
    gmap = {float(t): Fraction(float(gv)) for t, gv in zip(pts, g)}
    tq = [[1 / (Fraction(t) - xk) for xk in xf] for t in P]
    a = [[wk * tk for wk, tk in zip(wf, row)] for row in tq]
    idx = [(p, k) for p in range(len(P)) for k in range(n)]
    groups = [[a[p][k] * ff[k] for p, k in idx], [a[p][k] for p, k in idx],
              [a[p][k] for p, k in idx], [ff[k] * tq[p][k] for p, k in idx],
              [tq[p][k] for p, k in idx], [a[p][k] * ff[k] * tq[p][k] for p, k in idx],
              [a[p][k] * tq[p][k] for p, k in idx]]

    def adjoint(gr):
        NT, DT, DF, W1, W2, X1, X2 = gr
        df, dw, dx = [Fraction(0)] * n, [Fraction(0)] * n, [Fraction(0)] * n
        for p, t in enumerate(P):
            sl = slice(p * n, (p + 1) * n)
            Dp = sum(DT[sl])
            rp = sum(NT[sl]) / Dp
            cp = gmap[t] / Dp
            for k in range(n):
                i = p * n + k
                df[k] += cp * DF[i]
                dw[k] += cp * W1[i] - cp * rp * W2[i]
                dx[k] += cp * X1[i] - cp * rp * X2[i]
        return df + dw + dx

    sens = exact.term_sensitivities(adjoint, groups)
    pert = tuple(np.array([float(v) for v in sens[c * n:(c + 1) * n]]) for c in range(3))

    c_df, c_dw, c_dx = (np.zeros(n) for _ in range(3))
    for t in P:
        b = exact.blend_cardinals(x, d, Fraction(t))
        r = sum(bk * fk for bk, fk in zip(b, ff))
        lam = sum(abs(bk) for bk in b)
        sbf = sum(abs(bk * fk) for bk, fk in zip(b, ff))
        gp = abs(gmap[t])
        for k in range(n):
            tk = 1 / (Fraction(t) - xf[k])
            B = abs(ff[k]) + abs(r) + lam * abs(2 * r - ff[k]) + sbf
            c_df[k] += float(gp * abs(b[k]) * (1 + lam))
            c_dw[k] += float(gp * abs(b[k]) / abs(wf[k]) * B)
            c_dx[k] += float(gp * abs(b[k] * tk) * B)
    return pert, (c_df, c_dw, c_dx)


def weight_chain_abs(x, d):
    """A[k, l]: for the terms T_{k,i} = (-1)^i / prod_{j in window, j != k}
    (x_k - x_j) of w_k, the sum over i of the absolute values of the terms of
    d T_{k,i} / d x_l -- each by an exact central difference: for l != k the
    derivative in x_l; for l = k one derivative per factor, x_k moved in that
    factor alone (the terms an evaluation of d T / d x_k adds up)."""
    xf = _fr(x)
    n = len(xf)
    A = np.zeros((n, n))

    def term(k, i, moved=None, step=Fraction(0)):
        # moved = ("node", l): x_l moved everywhere; ("factor", j): x_k moved
        # in the factor of j only
        prod = Fraction(1)
        for j in range(i, i + d + 1):
            if j == k:
                continue
            xk, xj = xf[k], xf[j]
            if moved == ("node", j):
                xj += step
            if moved == ("factor", j):
                xk += step
            prod *= xk - xj
        return Fraction((-1) ** i) / prod

    for k in range(n):
        for i in range(max(0, k - d), min(k, n - 1 - d) + 1):
            for j in range(i, i + d + 1):
                if j == k:
                    continue
                for mv, col in ((("node", j), j), (("factor", j), k)):
                    dt = (term(k, i, mv, H) - term(k, i, mv, -H)) / (2 * H)
                    A[k, col] += float(abs(dt))
    return A


def check_grad_scales(scales, orc, x, f, d, pts, g):
    """scales = (s_df, s_dx, s_dn, s_dw, s_dxd) from one implementation of
    the adjoint's error scales.  Off-node terms against both exact routes,
    hit terms against the cardinal route, dL/dx_p against |g_p| S'
    (S' pinned by check_deriv_scale), and the chain part of s_dn against
    exact differences of the weight terms."""
    s_df, s_dx, s_dn, s_dw, s_dxd = (np.asarray(v, dtype=np.float64) for v in scales)
    w = orc.weights(x, d)
    pert, card = adjoint_scale_routes(x, f, w, d, pts, g)
    hit_df, hit_dx = np.zeros(x.size), np.zeros(x.size)
    for t, gv in zip(pts, g):
        j = np.flatnonzero(x == t)
        if j.size:
            hit_df[j[0]] += abs(gv)
            hit_dx[j[0]] += abs(gv) * float(node_deriv_scale(x, f, d, int(j[0])))
    lam_max = max([value_scale_routes(x, f, w, d, t)[2] for t in _non_hit_points(x, pts)] + [1.0])
    tol = 64 * U * (1 + lam_max) ** 2
    for name, got, pr, cr, hit in (("s_df", s_df, pert[0], card[0], hit_df),
                                   ("s_dw", s_dw, pert[1], card[1], 0.0),
                                   ("s_dxd", s_dxd, pert[2], card[2], hit_dx)):
        for ref, route in ((pr + hit, "perturbation"), (cr + hit, "cardinals")):
            err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
            assert np.all(err <= tol), (name, route, float(err.max()), tol)
    _, _, sd = orc.eval_deriv(x, f, d, pts)
    fin = np.isfinite(pts)
    ref_dx = np.where(fin, np.abs(g) * np.where(fin, sd, 0.0), 0.0)
    assert np.allclose(s_dx, ref_dx, rtol=1e-13, atol=0.0), ("s_dx", s_dx, ref_dx)
    ref = s_dxd + weight_chain_abs(x, d).T @ s_dw
    err = np.abs(s_dn - ref) / np.maximum(ref, 1e-300)
    assert np.all(err <= 16 * (d + 2) * U), ("s_dn chain", float(err.max()))
