// Fused second-form evaluation in binary64 (gfx950).
//
// For every point x and node k: delta = x - x_k, t = 1/delta,
//   N += (w_k f_k) t,   D += w_k t,   L += |w_k| |t|,
// then r = N / D and Lambda = L / |D| (Floater & Hormann 2007, barycentric
// form; Lambda is the Lebesgue function sum_k |a_k| / |sum_k a_k|).
//
// Mapping: each lane owns P points (strided by the block size so that the
// point loads and result stores are coalesced); all lanes of a wave walk the
// node table in the same order, so node records are wave-uniform and arrive
// through scalar loads as SGPR operands of the vector instructions.
//
// Reciprocals: a division costs far more than a multiply (the paper's
// premise for preferring scaling to quotients).  On gfx950 v_rcp_f64 is a
// quarter-rate estimate with about 25 correct bits.  Nodes are taken in
// groups of four and their reciprocals are formed from one reciprocal of the
// product (simultaneous inversion):
//   q01 = d0 d1, q23 = d2 d3, q = q01 q23, y ~ 1/q (rcp + one Newton step),
//   1/d0 = y q23 d1, 1/d1 = y q23 d0, 1/d2 = y q01 d3, 1/d3 = y q01 d2.
// Each t then carries a relative error of a few units in the last place,
// well inside the tolerance; the cost per pair drops from ~10 to ~7.75
// issue slots.
//
// Hits and range: q is zero exactly when some delta is zero (an exact hit),
// NaN for a NaN point, and infinite or subnormal only for extreme
// coordinates.  One v_cmp_class per group flags such lanes; after the node
// loop a flagged lane recomputes its point with one IEEE division per pair
// and the exact-hit branch (r = f_j bit-for-bit, Lambda = 1).  Unflagged
// lanes never branch inside the loop.
#include "fh_internal.h"

namespace fhk {

// true if v is +-0, subnormal, infinite or NaN (everything but normal)
__device__ __forceinline__ bool not_normal(double v) {
  return __builtin_amdgcn_class(v, 0x2F7);
}

// 1/q to ~2^-50 relative: hardware estimate plus one Newton step
__device__ __forceinline__ double rcp_refined(double q) {
  const double y = __builtin_amdgcn_rcp(q);
  const double e = __builtin_fma(-q, y, 1.0);
  return __builtin_fma(y, e, y);
}

// Exact per-pair evaluation of one point (flagged lanes only).
template <bool R, bool L>
__device__ __noinline__ void eval_point_exact(double t, const double* __restrict__ tx,
                                              const double* __restrict__ tw,
                                              const double* __restrict__ f, int64_t n,
                                              double* r_out, double* l_out) {
  double N = 0.0, D = 0.0, A = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double del = t - tx[k];
    if (del == 0.0) {
      *r_out = R ? f[k] : 0.0;
      *l_out = 1.0;
      return;
    }
    const double a = tw[k] / del;
    if (R) N = __builtin_fma(a, f[k], N);
    D = D + a;
    if (L) A = A + fabs(a);
  }
  *r_out = N / D;
  *l_out = A / fabs(D);
}

template <int P, bool R, bool L>
__global__ void __launch_bounds__(256)
    k_eval_f64(const double* __restrict__ x, int64_t m, const double* __restrict__ tx,
               const double* __restrict__ tw, const double* __restrict__ twf, int64_t n_pad,
               const double* __restrict__ f, int64_t n, double* __restrict__ r,
               double* __restrict__ lam) {
  const int64_t stride = blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * stride * P + threadIdx.x;
  double xp[P], N[P], D[P], A[P];
  bool bad[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * stride;
    xp[j] = x[idx < m ? idx : m - 1];
    N[j] = 0.0;
    D[j] = 0.0;
    A[j] = 0.0;
    bad[j] = false;
  }

#pragma unroll 2
  for (int64_t k = 0; k < n_pad; k += 4) {
    const double x0 = tx[k], x1 = tx[k + 1], x2 = tx[k + 2], x3 = tx[k + 3];
    const double w0 = tw[k], w1 = tw[k + 1], w2 = tw[k + 2], w3 = tw[k + 3];
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    if (R) {
      v0 = twf[k];
      v1 = twf[k + 1];
      v2 = twf[k + 2];
      v3 = twf[k + 3];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double d0 = xp[j] - x0, d1 = xp[j] - x1, d2 = xp[j] - x2, d3 = xp[j] - x3;
      const double q01 = d0 * d1, q23 = d2 * d3;
      const double q = q01 * q23;
      bad[j] |= not_normal(q);
      const double y = rcp_refined(q);
      const double y01 = y * q23, y23 = y * q01;
      const double t0 = y01 * d1, t1 = y01 * d0, t2 = y23 * d3, t3 = y23 * d2;
      D[j] = __builtin_fma(w0, t0, D[j]);
      D[j] = __builtin_fma(w1, t1, D[j]);
      D[j] = __builtin_fma(w2, t2, D[j]);
      D[j] = __builtin_fma(w3, t3, D[j]);
      if (R) {
        N[j] = __builtin_fma(v0, t0, N[j]);
        N[j] = __builtin_fma(v1, t1, N[j]);
        N[j] = __builtin_fma(v2, t2, N[j]);
        N[j] = __builtin_fma(v3, t3, N[j]);
      }
      if (L) {
        A[j] = __builtin_fma(fabs(w0), fabs(t0), A[j]);
        A[j] = __builtin_fma(fabs(w1), fabs(t1), A[j]);
        A[j] = __builtin_fma(fabs(w2), fabs(t2), A[j]);
        A[j] = __builtin_fma(fabs(w3), fabs(t3), A[j]);
      }
    }
  }

#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * stride;
    if (idx >= m) continue;
    double rv, lv;
    if (bad[j]) {
      eval_point_exact<R, L>(xp[j], tx, tw, f, n, &rv, &lv);
    } else {
      rv = N[j] / D[j];
      lv = A[j] / fabs(D[j]);
    }
    if (R) r[idx] = rv;
    if (L) lam[idx] = lv;
  }
}

template <int P>
static hipError_t launch_p(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                           double* lam, int block, hipStream_t s) {
  const int64_t per = (int64_t)block * P;
  const dim3 grid((unsigned)((m + per - 1) / per));
  if (r && lam)
    k_eval_f64<P, true, true><<<grid, block, 0, s>>>(x, m, t.x, t.w, t.wf, t.n_pad, t.f, n, r,
                                                     lam);
  else if (r)
    k_eval_f64<P, true, false><<<grid, block, 0, s>>>(x, m, t.x, t.w, t.wf, t.n_pad, t.f, n, r,
                                                      lam);
  else
    k_eval_f64<P, false, true><<<grid, block, 0, s>>>(x, m, t.x, t.w, t.wf, t.n_pad, t.f, n, r,
                                                      lam);
  return hipGetLastError();
}

hipError_t launch_eval_f64(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                           double* lam, const EvalConfig& cfg, hipStream_t s) {
  if (m == 0) return hipSuccess;
  switch (cfg.points_per_lane) {
    case 1: return launch_p<1>(x, m, t, n, r, lam, cfg.block, s);
    case 2: return launch_p<2>(x, m, t, n, r, lam, cfg.block, s);
    default: return launch_p<4>(x, m, t, n, r, lam, cfg.block, s);
  }
}

}  // namespace fhk
