/*
 * fh_oracle.c -- slow, plain binary64 reference implementation of
 * Floater-Hormann (FH) linear barycentric rational interpolation, its
 * Lebesgue function and the adjoint of r(x) with respect to the data.
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers. The product library
 * (HIP kernels behind the C ABI) shares no code, header, table or helper
 * with this file and never calls it.
 *
 * Sources of every formula:
 *   [FH]  M. S. Floater, K. Hormann, "Barycentric rational interpolation with
 *         no poles and high rates of approximation", Numer. Math. 107 (2007):
 *         the barycentric form r(x) = sum_k a_k(x) f_k / sum_k a_k(x) with
 *         a_k(x) = w_k / (x - x_k) and the weights
 *         w_k = sum_{i in J_k} (-1)^i prod_{j=i..i+d, j!=k} 1/(x_k - x_j),
 *         J_k = { i : max(0,k-d) <= i <= min(k, n-1-d) } (n nodes, 0-based).
 *   [LEB] The Lebesgue function of a linear interpolation scheme with
 *         cardinal functions b_k(x) = a_k(x) / sum_j a_j(x) is
 *         Lambda(x) = sum_k |b_k(x)| = sum_k |a_k(x)| / |sum_k a_k(x)|.
 *   [SW]  C. Schneider, W. Werner, "Some new aspects of rational
 *         interpolation", Math. Comp. 47 (1986): derivative of a barycentric
 *         rational at a node, r'(x_j) = sum_{k!=j} (w_k/w_j)(f_k - f_j)/(x_j - x_k).
 *   [NEU] A. Neumaier (1974): compensated summation (improved Kahan-Babuska).
 *   [LC]  The Lebesgue constant max_x Lambda(x) of an interpolation scheme,
 *         the quantity reported for FH by Bos, De Marchi, Hormann and Klein
 *         (Numer. Math. 2012); the search for it is a plain grid zoom.
 *   Paper (vector normalization, Mascarenhas): NaN propagation convention
 *         (Section 2, scaling algorithms propagate NaNs) and the IEEE rounding
 *         facts of the proofs appendix, in particular (rndA): multiplying a
 *         normal number by a power of two is exact.
 *
 * Conventions (readings where the sources are silent):
 *   - n nodes x_0 < x_1 < ... < x_{n-1}, strictly increasing and finite;
 *     0 <= d <= n-1.  Anything else is rejected with an error code.
 *   - An exact hit x == x_j (binary64 equality, so +0 == -0) returns
 *     r = f_j bit-for-bit and Lambda = 1.  NaN never hits.
 *   - A NaN point gives r = Lambda = NaN.  Infinite points are not special:
 *     every a_k is 0 and r = 0/0 = NaN.
 *   - Every quotient a_k = w_k/(x - x_k) is one IEEE division; every sum is
 *     taken in ascending k with Neumaier compensation, so the oracle is more
 *     accurate than any plain-summed evaluation it is compared with.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
  FHO_OK = 0,
  FHO_E_ARG = 1,
  FHO_E_DEGREE = 2,
  FHO_E_NODES = 3,
  FHO_E_NONFINITE = 4,
  FHO_E_RANGE = 5
};

/* ---------------------------------------------------------------- sums -- */
/* Neumaier's compensated sum: s holds the running sum, c the correction. */
typedef struct { double s, c; } csum;

static void cs_add(csum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}
static double cs_val(const csum* a) { return a->s + a->c; }

/* ----------------------------------------------------------- validation -- */
static int check_problem(const double* x, int64_t n, int32_t d) {
  if (n < 1 || x == NULL) return FHO_E_ARG;
  if (d < 0 || (int64_t)d > n - 1) return FHO_E_DEGREE;
  for (int64_t k = 0; k < n; ++k)
    if (!isfinite(x[k])) return FHO_E_NONFINITE;
  for (int64_t k = 0; k + 1 < n; ++k)
    if (!(x[k] < x[k + 1])) return FHO_E_NODES;
  return FHO_OK;
}

/* -------------------------------------------------------------- weights -- */
/* [FH] weights, literally: for each i in J_k the signed product of the
 * differences x_k - x_j over the window i..i+d without j = k, one division,
 * the factor (-1)^i, and the terms added in ascending i. */
int fho_weights(const double* x, int64_t n, int32_t d, double* w) {
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (w == NULL) return FHO_E_ARG;
  for (int64_t k = 0; k < n; ++k) {
    int64_t ilo = k - d > 0 ? k - d : 0;
    int64_t ihi = k < n - 1 - d ? k : n - 1 - d;
    double s = 0.0;
    for (int64_t i = ilo; i <= ihi; ++i) {
      double prod = 1.0;
      for (int64_t j = i; j <= i + d; ++j)
        if (j != k) prod = prod * (x[k] - x[j]);
      if (!isnormal(prod)) return FHO_E_RANGE;
      double term = 1.0 / prod;
      if (i % 2 != 0) term = -term;
      s = s + term;
    }
    if (!isnormal(s)) return FHO_E_RANGE;
    w[k] = s;
  }
  return FHO_OK;
}

/* Index j with x[j] == t, or -1 (binary search on strictly increasing x). */
static int64_t find_hit(const double* x, int64_t n, double t) {
  int64_t lo = 0, hi = n - 1;
  if (isnan(t)) return -1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (x[mid] == t) return mid;
    if (x[mid] < t)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

/* ------------------------------------------------------------ one point -- */
/* r(t), Lambda(t) and the error scale S(t) = sum|a_k f_k|/|D| + |r| Lambda,
 * used by the parity metric.  S is the largest first-order change of
 * r = N / D per unit relative error when every term of N = sum a_k f_k and of
 * D = sum a_k carries a relative error of its own (rounding of the terms and
 * of their sums, in any evaluation): with the cardinal functions
 * b_k = a_k / D, d r / d(N term k) = b_k f_k and d r / d(D term k) = -b_k r,
 * so S = sum|b_k f_k| + |r| sum|b_k|.  At a hit r = f_j is exact and S = |f_j|
 * only serves as a positive denominator.  compensated=0 gives the plain
 * ascending sum, reported only to show what compensation buys. */
static void eval_point(const double* x, const double* f, const double* w, int64_t n,
                       double t, int compensated, double* r, double* lam, double* scale) {
  if (isnan(t)) {
    *r = NAN; *lam = NAN; *scale = NAN;
    return;
  }
  int64_t j = find_hit(x, n, t);
  if (j >= 0) {
    *r = f[j]; *lam = 1.0; *scale = fabs(f[j]);
    return;
  }
  csum N = {0, 0}, D = {0, 0}, L = {0, 0}, A = {0, 0};
  double pn = 0, pd = 0, pl = 0, pa = 0;
  for (int64_t k = 0; k < n; ++k) {
    double a = w[k] / (t - x[k]);
    double p = a * f[k];
    if (compensated) {
      cs_add(&N, p); cs_add(&D, a); cs_add(&L, fabs(a)); cs_add(&A, fabs(p));
    } else {
      pn = pn + p; pd = pd + a; pl = pl + fabs(a); pa = pa + fabs(p);
    }
  }
  double nn = compensated ? cs_val(&N) : pn;
  double dd = compensated ? cs_val(&D) : pd;
  double ll = compensated ? cs_val(&L) : pl;
  double aa = compensated ? cs_val(&A) : pa;
  *r = nn / dd;
  *lam = ll / fabs(dd);
  *scale = aa / fabs(dd) + fabs(*r) * (*lam);
}

/* r (and optionally Lambda and S) at m points.  w may be NULL (computed
 * here).  nthreads <= 0 uses the OpenMP default.  The result does not
 * depend on the thread count. */
int fho_eval(const double* x, const double* f, int64_t n, int32_t d, const double* w_in,
             const double* pts, int64_t m, double* r, double* lam, double* scale,
             int32_t compensated, int32_t nthreads) {
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (f == NULL || m < 0 || (m > 0 && (pts == NULL || r == NULL))) return FHO_E_ARG;
  double* wbuf = NULL;
  const double* w = w_in;
  if (w == NULL) {
    wbuf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!wbuf) return FHO_E_ARG;
    st = fho_weights(x, n, d, wbuf);
    if (st != FHO_OK) { free(wbuf); return st; }
    w = wbuf;
  }
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int64_t p = 0; p < m; ++p) {
    double rr, ll, ss;
    eval_point(x, f, w, n, pts[p], compensated, &rr, &ll, &ss);
    r[p] = rr;
    if (lam) lam[p] = ll;
    if (scale) scale[p] = ss;
  }
  (void)nthreads;
  free(wbuf);
  return FHO_OK;
}

/* ---------------------------------------------------------- derivative -- */
/* r(x) and r'(x).  Away from the nodes r = N / D with N = sum a_k f_k,
   D = sum a_k (a_k = w_k / (x - x_k)); differentiating, N' = -F and D' = -E
   with F = sum a_k f_k / (x - x_k), E = sum a_k / (x - x_k), so
   r' = (N'D - N D') / D^2 = (r E - F) / D.  At a hit x == x_j the node
   formula of [SW]: r'(x_j) = sum_{k != j} (w_k / w_j)(f_k - f_j)/(x_j - x_k).
   A NaN or infinite point gives NaN for both.  The scale of the rounding
   error of r' is S', the largest first-order change of r' per unit relative
   error when every term of each of the four sums N, D, E, F carries a
   relative error of its own: with b_k = a_k / D, q_k = 1 / (x - x_k) and
   e = E / D = sum b_k q_k,
     d r' / d(N term k) = b_k f_k e,        d r' / d(D term k) = -b_k (r e + r'),
     d r' / d(E term k) = r b_k q_k,        d r' / d(F term k) = -b_k f_k q_k,
   so S' = |e| sum|b_k f_k| + |r e + r'| Lambda + sum|b_k q_k| (|r| + |f_k|).
   At a hit, S' = sum_{k != j} |w_k / w_j| |f_k - f_j| / |x_j - x_k|, the sum
   of the absolute values of the node formula's terms. */
static void deriv_point(const double* x, const double* f, const double* w, int64_t n, double t,
                        double* r, double* dr, double* scale) {
  if (!isfinite(t)) {
    *r = NAN; *dr = NAN; *scale = NAN;
    return;
  }
  int64_t j = find_hit(x, n, t);
  if (j >= 0) {
    csum s = {0, 0}, sa = {0, 0};
    for (int64_t k = 0; k < n; ++k) {
      if (k == j) continue;
      double term = (w[k] / w[j]) * (f[k] - f[j]) / (x[j] - x[k]);
      cs_add(&s, term);
      cs_add(&sa, fabs(term));
    }
    *r = f[j];
    *dr = cs_val(&s);
    *scale = cs_val(&sa);
    return;
  }
  csum N = {0, 0}, D = {0, 0}, E = {0, 0}, F = {0, 0};
  csum L = {0, 0}, A = {0, 0}, LQ = {0, 0}, FQ = {0, 0};
  for (int64_t k = 0; k < n; ++k) {
    double del = t - x[k];
    double a = w[k] / del;
    double q = 1.0 / del;
    double af = a * f[k];
    cs_add(&N, af);
    cs_add(&D, a);
    cs_add(&E, a * q);
    cs_add(&F, af * q);
    cs_add(&L, fabs(a));
    cs_add(&A, fabs(af));
    cs_add(&LQ, fabs(a * q));
    cs_add(&FQ, fabs(af * q));
  }
  double dd = cs_val(&D);
  double rr = cs_val(&N) / dd;
  double der = (rr * cs_val(&E) - cs_val(&F)) / dd;
  double lam = cs_val(&L) / fabs(dd);
  double e = cs_val(&E) / dd;
  *r = rr;
  *dr = der;
  *scale = fabs(e) * (cs_val(&A) / fabs(dd)) + fabs(rr * e + der) * lam +
           (fabs(rr) * cs_val(&LQ) + cs_val(&FQ)) / fabs(dd);
}

/* r and r' at m points (scale may be NULL); w may be NULL (computed here). */
int fho_eval_deriv(const double* x, const double* f, int64_t n, int32_t d, const double* w_in,
                   const double* pts, int64_t m, double* r, double* dr, double* scale,
                   int32_t nthreads) {
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (f == NULL || m < 0 || (m > 0 && (pts == NULL || r == NULL || dr == NULL))) return FHO_E_ARG;
  double* wbuf = NULL;
  const double* w = w_in;
  if (w == NULL) {
    wbuf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!wbuf) return FHO_E_ARG;
    st = fho_weights(x, n, d, wbuf);
    if (st != FHO_OK) { free(wbuf); return st; }
    w = wbuf;
  }
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int64_t p = 0; p < m; ++p) {
    double rr, dd, ss;
    deriv_point(x, f, w, n, pts[p], &rr, &dd, &ss);
    r[p] = rr;
    dr[p] = dd;
    if (scale) scale[p] = ss;
  }
  (void)nthreads;
  free(wbuf);
  return FHO_OK;
}

/* ---------------------------------------------------- Lebesgue constant -- */
/* Lambda(t) alone, summed as in eval_point (1 at a hit, NaN at a NaN point). */
static double lam_point(const double* x, const double* w, int64_t n, double t) {
  if (isnan(t)) return NAN;
  if (find_hit(x, n, t) >= 0) return 1.0;
  csum D = {0, 0}, L = {0, 0};
  for (int64_t k = 0; k < n; ++k) {
    double a = w[k] / (t - x[k]);
    cs_add(&D, a);
    cs_add(&L, fabs(a));
  }
  return cs_val(&L) / fabs(cs_val(&D));
}

/* [LC] The Lebesgue constant of the scheme is the largest value of its
 * Lebesgue function on [x_0, x_{n-1}]; Lambda = 1 at the nodes, so it is
 * the largest of the maxima over the n-1 intervals [x_k, x_{k+1}].  Each
 * interval's maximum is searched for by sampling and zooming in:
 *   a round samples S interior points of the current bracket [lo, hi],
 *     h = (hi - lo) / (S + 1),  t_i = lo + (i + 1) h,  i = 0..S-1
 *   (the product (i + 1) h and the sum rounded separately);
 *   i* is the first index of the largest sampled Lambda (NaN never counts;
 *   if every sample is NaN the search of this interval stops);
 *   the next round's bracket is [t_{i*-1}, t_{i*+1}] with t_{-1} = lo and
 *   t_S = hi; the first round's bracket is the interval itself.
 * After R rounds lam_out[k] is the largest Lambda seen in any round (the
 * first seen on ties) and x_out[k] the sample where it was seen (NaN, NaN
 * if none was a number).  The search converges to the interval's maximum
 * when Lambda has one local maximum there (true of the FH node families
 * this is used with); each round divides the bracket by (S + 1) / 2. */
int fho_lebesgue_max(const double* x, int64_t n, int32_t d, const double* w_in, int32_t samples,
                     int32_t rounds, const int64_t* ks, int64_t nk, double* lam_out,
                     double* x_out, int32_t nthreads) {
  /* ks: the intervals to search (nk of them, outputs in that order), or
     NULL for all n - 1 */
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (ks == NULL) nk = n - 1;
  if (samples < 1 || rounds < 1 || nk < 0 || (nk > 0 && (lam_out == NULL || x_out == NULL)))
    return FHO_E_ARG;
  for (int64_t q = 0; ks != NULL && q < nk; ++q)
    if (ks[q] < 0 || ks[q] >= n - 1) return FHO_E_ARG;
  double* wbuf = NULL;
  const double* w = w_in;
  if (w == NULL) {
    wbuf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!wbuf) return FHO_E_ARG;
    st = fho_weights(x, n, d, wbuf);
    if (st != FHO_OK) { free(wbuf); return st; }
    w = wbuf;
  }
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
  for (int64_t q = 0; q < nk; ++q) {
    int64_t k = ks != NULL ? ks[q] : q;
    double lo = x[k], hi = x[k + 1];
    double best = -INFINITY, best_x = NAN;
    for (int32_t r = 0; r < rounds; ++r) {
      double h = (hi - lo) / (double)(samples + 1);
      int32_t bi = -1;
      double bv = -INFINITY;
      for (int32_t i = 0; i < samples; ++i) {
        double t = lo + (double)(i + 1) * h;
        double v = lam_point(x, w, n, t);
        if (v > bv) { bv = v; bi = i; }
      }
      if (bi < 0) break;
      double t_best = lo + (double)(bi + 1) * h;
      if (bv > best) { best = bv; best_x = t_best; }
      double nlo = bi > 0 ? lo + (double)bi * h : lo;
      double nhi = bi < samples - 1 ? lo + (double)(bi + 2) * h : hi;
      lo = nlo;
      hi = nhi;
    }
    lam_out[q] = best == -INFINITY ? NAN : best;
    x_out[q] = best == -INFINITY ? NAN : best_x;
  }
  (void)nthreads;
  free(wbuf);
  return FHO_OK;
}

/* Number of threads fho_eval would use for a given request. */
int fho_threads(int32_t nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* ------------------------------------------------------------- adjoint -- */
/* Loss L = sum_p g_p r(x_p).  Outputs (any may be NULL):
 *   df[k]  = dL/df_k
 *   dpt[p] = dL/dx_p
 *   dw[k]  = dL/dw_k            (weights held fixed)
 *   dxk[k] = dL/dx_k            (total: direct term plus the chain through w)
 * Formulas at a non-hit point, with a_k = w_k/(x-x_k), D = sum a_k, r = N/D:
 *   dr/df_k = a_k / D
 *   dr/dx   = sum_k a_k (r - f_k) / (x - x_k) / D
 *   dr/dw_k = (f_k - r) / ((x - x_k) D)
 *   dr/dx_k |_w = a_k (f_k - r) / ((x - x_k) D)
 * A NaN or infinite point has no derivative: dL/dx_p = NaN and the point
 * contributes nothing to the other gradients.
 * At a hit x == x_j: r = f_j whatever the weights, so dr/df_j = 1, dr/dw = 0,
 * dr/dx_k|_w = 0 for k != j, dr/dx = r'(x_j) by [SW], and
 * dr/dx_j|_w = -r'(x_j) because r depends on the nodes only through x - x_k.
 * The chain through the weights uses, for the term
 *   T_{k,i} = (-1)^i / prod_{j in [i,i+d], j!=k} (x_k - x_j),
 *   dT/dx_l = T / (x_k - x_l) for l != k in the window,
 *   dT/dx_k = -T * sum_{l in window, l!=k} 1 / (x_k - x_l).
 * Per-node sums over points are accumulated in fixed chunks of points, each
 * chunk with compensated sums, and the chunks are added in order, so the
 * result does not depend on the thread count. */
#define FHO_CHUNKS 64

int fho_backward(const double* x, const double* f, int64_t n, int32_t d, const double* pts,
                 int64_t m, const double* g, double* df, double* dpt, double* dw, double* dxk,
                 int32_t nthreads) {
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (f == NULL || m < 0 || (m > 0 && (pts == NULL || g == NULL))) return FHO_E_ARG;
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  if (!w) return FHO_E_ARG;
  st = fho_weights(x, n, d, w);
  if (st != FHO_OK) { free(w); return st; }

  /* per chunk, per node: compensated sums of dL/df, dL/dw, dL/dx_k|_w */
  size_t per = (size_t)n * 3;
  csum* acc = (csum*)calloc((size_t)FHO_CHUNKS * per, sizeof(csum));
  if (!acc) { free(w); return FHO_E_ARG; }

#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int c = 0; c < FHO_CHUNKS; ++c) {
    int64_t p0 = m * c / FHO_CHUNKS, p1 = m * (c + 1) / FHO_CHUNKS;
    csum* a_df = acc + (size_t)c * per;
    csum* a_dw = a_df + n;
    csum* a_dx = a_dw + n;
    for (int64_t p = p0; p < p1; ++p) {
      double t = pts[p], gp = g[p];
      /* r is not differentiable at a non-finite point: dL/dx_p is NaN and
         the point adds nothing to the node gradients */
      if (!isfinite(t)) {
        if (dpt) dpt[p] = NAN;
        continue;
      }
      int64_t j = find_hit(x, n, t);
      if (j >= 0) {
        /* r'(x_j) by [SW] */
        csum s = {0, 0};
        for (int64_t k = 0; k < n; ++k)
          if (k != j) cs_add(&s, (w[k] / w[j]) * (f[k] - f[j]) / (x[j] - x[k]));
        double rp = cs_val(&s);
        cs_add(&a_df[j], gp);
        cs_add(&a_dx[j], -gp * rp);
        if (dpt) dpt[p] = gp * rp;
        continue;
      }
      csum N = {0, 0}, D = {0, 0};
      for (int64_t k = 0; k < n; ++k) {
        double a = w[k] / (t - x[k]);
        cs_add(&N, a * f[k]);
        cs_add(&D, a);
      }
      double dd = cs_val(&D);
      double rr = cs_val(&N) / dd;
      csum S = {0, 0};
      for (int64_t k = 0; k < n; ++k) {
        double del = t - x[k];
        double a = w[k] / del;
        double e = (f[k] - rr) / (del * dd); /* dr/dw_k */
        cs_add(&S, -a * e);                  /* a_k (r - f_k)/((x-x_k) D) */
        cs_add(&a_df[k], gp * (a / dd));
        cs_add(&a_dw[k], gp * e);
        cs_add(&a_dx[k], gp * a * e);
      }
      if (dpt) dpt[p] = gp * cs_val(&S);
    }
  }

  /* reduce the chunks in order */
  double* sdf = (double*)malloc(sizeof(double) * (size_t)n * 3);
  if (!sdf) { free(acc); free(w); return FHO_E_ARG; }
  double* sdw = sdf + n;
  double* sdx = sdw + n;
  for (int64_t k = 0; k < n; ++k) {
    csum t0 = {0, 0}, t1 = {0, 0}, t2 = {0, 0};
    for (int c = 0; c < FHO_CHUNKS; ++c) {
      const csum* b = acc + (size_t)c * per;
      cs_add(&t0, cs_val(&b[k]));
      cs_add(&t1, cs_val(&b[n + k]));
      cs_add(&t2, cs_val(&b[2 * n + k]));
    }
    sdf[k] = cs_val(&t0);
    sdw[k] = cs_val(&t1);
    sdx[k] = cs_val(&t2);
  }
  free(acc);

  if (df) memcpy(df, sdf, sizeof(double) * (size_t)n);
  if (dw) memcpy(dw, sdw, sizeof(double) * (size_t)n);
  if (dxk) {
    /* chain through the weights: dL/dx_l += sum_k dL/dw_k dw_k/dx_l */
    csum* tot = (csum*)calloc((size_t)n, sizeof(csum));
    if (!tot) { free(sdf); free(w); return FHO_E_ARG; }
    for (int64_t l = 0; l < n; ++l) cs_add(&tot[l], sdx[l]);
    for (int64_t k = 0; k < n; ++k) {
      int64_t ilo = k - d > 0 ? k - d : 0;
      int64_t ihi = k < n - 1 - d ? k : n - 1 - d;
      for (int64_t i = ilo; i <= ihi; ++i) {
        double prod = 1.0;
        for (int64_t j = i; j <= i + d; ++j)
          if (j != k) prod = prod * (x[k] - x[j]);
        double T = 1.0 / prod;
        if (i % 2 != 0) T = -T;
        csum sk = {0, 0};
        for (int64_t l = i; l <= i + d; ++l) {
          if (l == k) continue;
          double q = T / (x[k] - x[l]);
          cs_add(&tot[l], sdw[k] * q);
          cs_add(&sk, q);
        }
        cs_add(&tot[k], -sdw[k] * cs_val(&sk));
      }
    }
    for (int64_t l = 0; l < n; ++l) dxk[l] = cs_val(&tot[l]);
    free(tot);
  }
  free(sdf);
  free(w);
  return FHO_OK;
}

/* Error scales of the adjoint: for every gradient component, the largest
   first-order change per unit relative error when every term that an
   evaluation of the adjoint forms carries a relative error of its own:
   per point the terms of N_p = sum a_pk f_k and D_p = sum a_pk (through
   r_p = N_p / D_p and c_p = g_p / D_p), and per node the terms of the
   node sums over points, c_p a_pk (dL/df_k), c_p f_k t_pk and c_p r_p t_pk
   (dL/dw_k), c_p a_pk f_k t_pk and c_p a_pk r_p t_pk (dL/dx_k at fixed
   weights), t_pk = 1 / (x_p - x_k).  With b_k = a_pk / D_p, Lambda_p and
   B_pk = |f_k| + |r_p| + Lambda_p |2 r_p - f_k| + sum_j |b_j f_j|:
     s_df[k] = sum_p |g_p b_k| (1 + Lambda_p),
     s_dw[k] = sum_p |c_p t_pk| B_pk,    s_dxd[k] = sum_p |g_p b_k t_pk| B_pk,
     s_dx[p] = |g_p| S'(x_p) (S' the derivative's scale; dL/dx_p = g_p r'),
   and s_dn[l] = s_dxd[l] + sum_k s_dw[k] sum_{i in J_k} |d T_{k,i} / d x_l|
   for the total node gradient (the chain through the weights).  At a hit
   x_p == x_j: |g_p| goes to s_df[j], |g_p| S'(x_j) to s_dx[p] and to s_dxd[j].
   A non-finite point adds nothing (s_dx = 0).  Plain sums over points:
   these are tolerances, not results.  s_dw and s_dxd (may be NULL) return
   the two parts of s_dn. */
int fho_grad_scales(const double* x, const double* f, int64_t n, int32_t d, const double* pts,
                    int64_t m, const double* g, double* s_df, double* s_dx, double* s_dn,
                    double* s_dw, double* s_dxd, int32_t nthreads) {
  int st = check_problem(x, n, d);
  if (st != FHO_OK) return st;
  if (f == NULL || m < 0 || (m > 0 && (pts == NULL || g == NULL))) return FHO_E_ARG;
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  if (!w) return FHO_E_ARG;
  st = fho_weights(x, n, d, w);
  if (st != FHO_OK) { free(w); return st; }
  size_t per = (size_t)n * 3;
  double* acc = (double*)calloc((size_t)FHO_CHUNKS * per, sizeof(double));
  if (!acc) { free(w); return FHO_E_ARG; }

#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int c = 0; c < FHO_CHUNKS; ++c) {
    int64_t p0 = m * c / FHO_CHUNKS, p1 = m * (c + 1) / FHO_CHUNKS;
    double* a_df = acc + (size_t)c * per;
    double* a_dw = a_df + n;
    double* a_dx = a_dw + n;
    for (int64_t p = p0; p < p1; ++p) {
      double t = pts[p], gp = fabs(g[p]);
      if (s_dx) s_dx[p] = 0.0;
      if (!isfinite(t)) continue;
      double rr, der, sd;
      deriv_point(x, f, w, n, t, &rr, &der, &sd);
      if (s_dx) s_dx[p] = gp * sd;
      int64_t j = find_hit(x, n, t);
      if (j >= 0) {
        a_df[j] += gp;
        a_dx[j] += gp * sd;
        continue;
      }
      csum D = {0, 0}, L = {0, 0}, A = {0, 0};
      for (int64_t k = 0; k < n; ++k) {
        double a = w[k] / (t - x[k]);
        cs_add(&D, a);
        cs_add(&L, fabs(a));
        cs_add(&A, fabs(a * f[k]));
      }
      double dd = fabs(cs_val(&D));
      double lam = cs_val(&L) / dd, sbf = cs_val(&A) / dd, cp = gp / dd;
      for (int64_t k = 0; k < n; ++k) {
        double q = 1.0 / fabs(t - x[k]);
        double bk = fabs(f[k]) + fabs(rr) + lam * fabs(2.0 * rr - f[k]) + sbf;
        a_df[k] += fabs(w[k]) * cp * q * (1.0 + lam);
        a_dw[k] += cp * q * bk;
        a_dx[k] += fabs(w[k]) * cp * q * q * bk;
      }
    }
  }

  double* sw = (double*)calloc((size_t)n, sizeof(double));
  if (!sw) { free(acc); free(w); return FHO_E_ARG; }
  for (int64_t k = 0; k < n; ++k) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int c = 0; c < FHO_CHUNKS; ++c) {
      const double* b = acc + (size_t)c * per;
      t0 += b[k];
      t1 += b[n + k];
      t2 += b[2 * n + k];
    }
    if (s_df) s_df[k] = t0;
    sw[k] = t1;
    if (s_dw) s_dw[k] = t1;
    if (s_dxd) s_dxd[k] = t2;
    if (s_dn) s_dn[k] = t2;
  }
  free(acc);
  if (s_dn) {
    for (int64_t k = 0; k < n; ++k) {
      int64_t ilo = k - d > 0 ? k - d : 0;
      int64_t ihi = k < n - 1 - d ? k : n - 1 - d;
      for (int64_t i = ilo; i <= ihi; ++i) {
        double prod = 1.0;
        for (int64_t j = i; j <= i + d; ++j)
          if (j != k) prod = prod * fabs(x[k] - x[j]);
        double T = 1.0 / prod, inv = 0.0;
        for (int64_t l = i; l <= i + d; ++l) {
          if (l == k) continue;
          s_dn[l] += sw[k] * T / fabs(x[k] - x[l]);
          inv += 1.0 / fabs(x[k] - x[l]);
        }
        s_dn[k] += sw[k] * T * inv;
      }
    }
  }
  free(sw);
  free(w);
  return FHO_OK;
}
