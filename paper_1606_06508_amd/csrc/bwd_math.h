// Binary64 pieces of the adjoint shared by the binary64 and precision-split
// kernels: the pair-by-pair treatment of one point (exact hits, extreme
// range) and of one (point, node) pair in the per-node pass.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pair_math.h"

namespace fhk {

constexpr int kPartFields = 6;  // S1, S2, S3, S4, H1 (sum g_hit), H2 (sum g_hit r')

// Per-point records written by the point pass and read by the node pass,
// one array per field ([m_pad] each), so that the node pass reads a group
// of consecutive points with one wide scalar load per field.
struct PointRecs {
  double* x;    // the point (a far point for padding and non-finite points)
  double* c;    // c = g / D (0 at hits)
  double* cr;   // c r
  double* hg;   // g at a hit, else 0
  double* hgr;  // g r'(x_j) at a hit, else 0
};

// Point x (finite) with loss weight gp, nodes tx/tw/tf[0, n), by one IEEE
// division per pair.  At a hit x == x_j: r = f_j whatever the weights, so
// the point's weight goes to the hit sums (hg = g, hgr = g r'(x_j), node
// derivative of Schneider & Werner 1986) and c = c r = 0.  Otherwise
// c = g / D, c r and dx = c (r E - F) from the plain sums.  *r_val (if
// given) receives r.
__device__ inline void bwd_point_exact(double x, double gp, const double* __restrict__ tx,
                                       const double* __restrict__ tw,
                                       const double* __restrict__ tf, int64_t n, double* dxp,
                                       double* c, double* cr, double* hg, double* hgr,
                                       double* r_val = nullptr) {
  // the hit by binary search, then loops without early exits (their loads
  // pipeline; a flagged lane holds its whole wave)
  const int64_t hit = find_node(x, tx, n);
  double n2 = 0.0, d2 = 0.0, e2 = 0.0, f2 = 0.0;
#pragma unroll 4
  for (int64_t k = 0; hit < 0 && k < n; ++k) {
    const double del = x - tx[k];
    const double a = tw[k] / del;
    const double q = 1.0 / del;
    d2 += a;
    n2 = __builtin_fma(a, tf[k], n2);
    e2 = __builtin_fma(a, q, e2);
    f2 = __builtin_fma(a * tf[k], q, f2);
  }
  if (hit >= 0) {
    const double wj = tw[hit], fj = tf[hit], xj = tx[hit];
    double rp = 0.0;
#pragma unroll 4
    for (int64_t k = 0; k < n; ++k)
      if (k != hit) rp += (tw[k] / wj) * (tf[k] - fj) / (xj - tx[k]);
    *dxp = gp * rp;
    *c = 0.0;
    *cr = 0.0;
    *hg = gp;
    *hgr = gp * rp;
    if (r_val) *r_val = fj;
  } else {
    const double r = n2 / d2;
    if (r_val) *r_val = r;
    *c = gp / d2;
    *cr = *c * r;
    *dxp = *c * (r * e2 - f2);
    *hg = 0.0;
    *hgr = 0.0;
  }
}

// One (point p, node xk) pair of the per-node pass by IEEE division; a zero
// difference is a hit of the point on this node.  FULL: all sums, else S1
// and H1 only (the node gradient is not wanted).
template <bool FULL = true>
__device__ inline void bwd_pair_exact(const PointRecs& rec, int64_t p, double xk, double& S1,
                                      double& S2, double& S3, double& S4, double& H1,
                                      double& H2) {
  const double dl = rec.x[p] - xk;
  if (dl == 0.0) {
    H1 += rec.hg[p];
    if (FULL) H2 += rec.hgr[p];
  } else {
    const double ti = 1.0 / dl;
    S1 = __builtin_fma(rec.c[p], ti, S1);
    if (FULL) {
      const double t2 = ti * ti;
      S2 = __builtin_fma(rec.cr[p], ti, S2);
      S3 = __builtin_fma(rec.c[p], t2, S3);
      S4 = __builtin_fma(rec.cr[p], t2, S4);
    }
  }
}

}  // namespace fhk
