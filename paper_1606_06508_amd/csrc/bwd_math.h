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

// One (point, node xk) pair of the per-node pass by IEEE division, from the
// point's record {x, c, c r, g at a hit, g r'(x_j) at a hit}; a zero
// difference is a hit of the point on this node.  SUMS: 2 all node sums,
// 1 S1 and H1 only (the node gradient is not wanted), 0 none.  PT: the
// point-side term (w_k r_p - w_k f_k) t^2 of dL/dx_p / c_p is added to gp
// (rp = r_p; nothing at a hit).
template <int SUMS = 2, bool PT = false>
__device__ inline void bwd_pair_exact(double px, double pc, double pcr, double phg, double phgr,
                                      double xk, double& S1, double& S2, double& S3, double& S4,
                                      double& H1, double& H2, double wk = 0.0, double wfk = 0.0,
                                      double rp = 0.0, double* gp = nullptr) {
  const double dl = px - xk;
  if (dl == 0.0) {
    if (SUMS >= 1) H1 += phg;
    if (SUMS == 2) H2 += phgr;
  } else {
    const double ti = 1.0 / dl;
    if (SUMS >= 1) S1 = __builtin_fma(pc, ti, S1);
    if (SUMS == 2 || PT) {
      const double t2 = ti * ti;
      if (SUMS == 2) {
        S2 = __builtin_fma(pcr, ti, S2);
        S3 = __builtin_fma(pc, t2, S3);
        S4 = __builtin_fma(pcr, t2, S4);
      }
      if (PT) *gp = __builtin_fma(__builtin_fma(wk, rp, -wfk), t2, *gp);
    }
  }
}

// ---- sums across the 64 lanes of a wave ----
// A DPP lane move inside 16-lane rows (every source lane valid); binary64
// values move as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u)), CTRL,
                                             0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u >> 32)),
                                             CTRL, 0xf, 0xf, false);
  return __longlong_as_double(static_cast<long long>(
      (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo)));
}

// Orders this wave's LDS accesses across lanes (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Transposed wave sum of eight values per lane through the wave's own
// 4 KB of LDS (lds[8][64]): afterwards lane l holds the sum over all 64
// lanes of v[l >> 3] (the same bits on its group of eight lanes), in a fixed
// order: lane l adds the values of lanes 8 (l & 7) .. 8 (l & 7) + 7 in
// order, then the eight lanes of the group combine by DPP (quad_perm xor 1,
// xor 2, row_half_mirror).  Eight LDS stores, four 16-byte loads and 16
// VALU instructions per call.
__device__ __forceinline__ double wave_sum8(const double (&v)[8], double* lds) {
  const int lane = threadIdx.x & 63;
  wave_lds_sync();  // the previous call's loads are done
#pragma unroll
  for (int j = 0; j < 8; ++j) lds[j * 64 + lane] = v[j];
  wave_lds_sync();
  const double2* src = reinterpret_cast<const double2*>(lds + (lane >> 3) * 64 + (lane & 7) * 8);
  double z = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double2 q = src[r];
    z = r == 0 ? q.x + q.y : (z + q.x) + q.y;
  }
  z += dpp_f64<0xB1>(z);   // quad_perm [1,0,3,2]
  z += dpp_f64<0x4E>(z);   // quad_perm [2,3,0,1]
  z += dpp_f64<0x141>(z);  // row_half_mirror
  return z;
}

}  // namespace fhk
