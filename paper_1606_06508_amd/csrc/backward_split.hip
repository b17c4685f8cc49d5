// Precision-split adjoint (gfx950): binary32 pair terms, binary64 data and
// accumulators, the same arithmetic contract as the split evaluation.
//
// Pass 1 (lanes own points; node records {x head, x tail, w 2^-e,
// w f 2^-ef} staged in LDS): binary32 tile sums of D, N, E = sum w t^2 and
// F = sum w f t^2 over kTile nodes, promoted to binary64; then
// r = 2^(ef-e) N / D and dL/dx_p = (g / D)(r E - 2^(ef-e) F) with D, E, N, F
// the scaled sums.  The pass-2 record carries c 2^e = g / D (scaled D), which
// stays near the scale of g whatever the scale of the weights; pass 3
// removes the factor exactly.
//
// Pass 2 (lanes own nodes; point records {x head, x tail, c 2^e, c r 2^e} in
// binary32 staged in LDS): binary32 tile sums of S1..S4 over kTile points,
// promoted to binary64.  A lane whose tile sums are not finite (a point on
// its node gives t = inf; some records force it, below) redoes that tile
// pair by pair with binary64 sums.
//
// Differences are float-float, (x_hi - k_hi) + (x_lo - k_lo), with the same
// operations in both passes, so a pair gets the same t in both; reciprocals
// are v_rcp_f32.  Next to a node the float-float difference is off by up to
// 2^-48 |x| absolute, which is harmless as long as c_p and the pair terms
// use the same t: the result is then the exact gradient for a point moved
// by that much.  So the redo must use, for each point, the reciprocal its c
// was computed with: the binary32 one for points whose c comes from the
// binary32 sums of pass 1, the binary64 one (and the exact-hit test) for
// points that pass 1 sent to the binary64 per-pair path.  The binary32
// record says which:
//   {head, tail, c, c r}    binary32 c, usable by the binary32 sums;
//   {head, tail, NaN, NaN}  binary32 c out of the binary32 range (below):
//                           binary64 sums with the binary32 reciprocal;
//   {NaN, NaN, 0, 0}        binary64 c: binary64 sums and reciprocal;
//   {head, tail, 0, 0}      no weight (hits, padding, non-finite points):
//                           only an exact hit on the node adds anything.
//
// Range.  The evaluation's binary32 domain applies (node span, weight
// ranges, points within one span of the nodes; see split_math.h), with the
// binary32 record usable only when c 2^e and c r 2^e are zero or of
// magnitude in [2^-50, 2^50]: then, as |t| >= 2^-22, every binary32 term is
// normal or overflows, and overflow is caught by the finiteness check.
#include "bwd_math.h"
#include "fh_internal.h"
#include "split_math.h"

namespace fhk {

__device__ __forceinline__ bool in_binary32_range(double v) {
  const double a = fabs(v);
  return v == 0.0 || (a >= 0x1p-50 && a <= 0x1p50);
}

// ---------------------------------------------------------------- pass 1 --
// DERIV: write r (r_out) and the derivative r' (dx) only, as if g_p = 1;
// no records (m_pad = m).  EF: E and F are summed (for dx).  SAVE (with EF,
// not DERIV): the forward of the saved-state adjoint -- r, r' and the
// records for g_p = 1 with r in place of c r, and in rec32 {head, tail,
// 1 if the point took the binary64 path else 0, 0}, from which
// k_bwd_scale_records_split builds the records for the loss weights.
template <int P, bool DERIV, bool EF, bool SAVE = false>
__global__ void __launch_bounds__(kStage)
    k_bwd_points_split(const double* __restrict__ x, const double* __restrict__ g, int64_t m,
                       int64_t m_pad, const float4* __restrict__ s4, int64_t n_pad,
                       const double* __restrict__ tx, const double* __restrict__ tw,
                       const double* __restrict__ tf, int64_t n,
                       const int32_t* __restrict__ scale_exp, double* __restrict__ dx,
                       PointRecs rec, float4* __restrict__ rec32, double* __restrict__ r_out) {
  __shared__ float4 stage[2][kStage];
  const int64_t base = (int64_t)blockIdx.x * kStage * P + threadIdx.x;
  const double x_first = tx[0], x_last = tx[n - 1];
  const double span = x_last - x_first;
  // a point far outside the node range: its differences are all >= 1
  const double far = x_last + span + 1.0;
  double xp[P], N[P], D[P], E[P], F[P];
  float xh[P], xl[P], Nt[P], Dt[P], Et[P], Ft[P];
  bool bad[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + (int64_t)j * kStage;
    xp[j] = idx < m ? x[idx] : far;
    xh[j] = (float)xp[j];
    xl[j] = (float)(xp[j] - (double)xh[j]);
    N[j] = D[j] = E[j] = F[j] = 0.0;
    Nt[j] = Dt[j] = Et[j] = Ft[j] = 0.0f;
    bad[j] = idx < m && !in_split_domain(xp[j], x_first, x_last);
  }

  staged_tiles(
      stage, s4, n_pad,
      [&](const float4(&rc)[4]) {
        float t[4][P];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) t[q][j] = (xh[j] - rc[q].x) + (xl[j] - rc[q].y);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) t[q][j] = __builtin_amdgcn_rcpf(t[q][j]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) {
            Dt[j] = __builtin_fmaf(rc[q].z, t[q][j], Dt[j]);
            Nt[j] = __builtin_fmaf(rc[q].w, t[q][j], Nt[j]);
            if constexpr (EF) {
              const float t2 = t[q][j] * t[q][j];
              Et[j] = __builtin_fmaf(rc[q].z, t2, Et[j]);
              Ft[j] = __builtin_fmaf(rc[q].w, t2, Ft[j]);
            }
          }
      },
      [&](int64_t, int64_t) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          bad[j] |= not_finite32(Dt[j]) | not_finite32(Nt[j]);
          D[j] += (double)Dt[j];
          N[j] += (double)Nt[j];
          Dt[j] = Nt[j] = 0.0f;
          if constexpr (EF) {
            bad[j] |= not_finite32(Et[j]) | not_finite32(Ft[j]);
            E[j] += (double)Et[j];
            F[j] += (double)Ft[j];
            Et[j] = Ft[j] = 0.0f;
          }
        }
      });

  const int e = scale_exp[0], shift = scale_exp[1];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + (int64_t)j * kStage;
    if (idx >= m_pad) continue;
    double xr = xp[j], c = 0.0, cr = 0.0, hg = 0.0, hgr = 0.0;
    if (idx < m) {
      const double gp = (DERIV || SAVE) ? 1.0 : g[idx];
      double dxp, rv;
      if (!__builtin_isfinite(xp[j])) {
        dxp = rv = __builtin_nan("");
        xr = far;
      } else if (!bad[j]) {
        rv = ldexp(N[j] / D[j], shift);
        c = gp / D[j];  // = 2^e g / D_p
        cr = c * rv;
        dxp = EF ? c * (rv * E[j] - ldexp(F[j], shift)) : 0.0;
      } else {
        bwd_point_exact(xp[j], gp, tx, tw, tf, n, &dxp, &c, &cr, &hg, &hgr, &rv);
        c = ldexp(c, e);
        cr = ldexp(cr, e);
      }
      if (EF && dx) dx[idx] = dxp;
      if ((DERIV || SAVE) && r_out) r_out[idx] = rv;
      if (SAVE) cr = rv;
    }
    if (DERIV) continue;
    rec.x[idx] = xr; rec.c[idx] = c; rec.cr[idx] = cr; rec.hg[idx] = hg; rec.hgr[idx] = hgr;
    const float h = (float)xr, l = (float)(xr - (double)h), nan = __builtin_nanf("");
    if (SAVE) {
      rec32[idx] = make_float4(h, l, bad[j] ? 1.0f : 0.0f, 0.0f);
      continue;
    }
    float4 r32;
    if (c == 0.0 && cr == 0.0)
      r32 = make_float4(h, l, 0.0f, 0.0f);
    else if (bad[j])
      r32 = make_float4(nan, nan, 0.0f, 0.0f);
    else if (in_binary32_range(c) && in_binary32_range(cr))
      r32 = make_float4(h, l, (float)c, (float)cr);
    else
      r32 = make_float4(h, l, nan, nan);
    rec32[idx] = r32;
  }
}

// Saved-state adjoint, before pass 2: the records for the loss weights g
// from the forward's records for g = 1 (saved, saved32; see SAVE above; the
// point coordinates rec.x are shared): c = g c1, c r, g and g r'(x_j) at a
// hit, and the binary32 record coded as pass 1 codes it.
__global__ void __launch_bounds__(256)
    k_bwd_scale_records_split(PointRecs saved, const float4* __restrict__ saved32,
                              const double* __restrict__ g, int64_t m, int64_t m_pad,
                              PointRecs rec, float4* __restrict__ rec32) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m_pad) return;
  const double gp = p < m ? g[p] : 0.0;
  const double c1 = saved.c[p];
  const bool hit = saved.hg[p] != 0.0;
  const double c = c1 == 0.0 ? 0.0 : gp * c1;
  const double cr = c1 == 0.0 ? 0.0 : c * saved.cr[p];
  rec.c[p] = c;
  rec.cr[p] = cr;
  rec.hg[p] = hit ? gp : 0.0;
  rec.hgr[p] = hit ? gp * saved.hgr[p] : 0.0;
  const float4 s32 = saved32[p];
  const float nan = __builtin_nanf("");
  float4 r32;
  if (c == 0.0 && cr == 0.0)
    r32 = make_float4(s32.x, s32.y, 0.0f, 0.0f);
  else if (s32.z != 0.0f)
    r32 = make_float4(nan, nan, 0.0f, 0.0f);
  else if (in_binary32_range(c) && in_binary32_range(cr))
    r32 = make_float4(s32.x, s32.y, (float)c, (float)cr);
  else
    r32 = make_float4(s32.x, s32.y, nan, nan);
  rec32[p] = r32;
}

// ---------------------------------------------------------------- pass 2 --
// grid: x = node tiles of kStage * Q nodes (lane l of the block owns nodes
// l, l + kStage, ...), y = chunks of `chunk` points (a multiple of kTile).
// FULL: all four sums and both hit sums (the node gradient needs them);
// otherwise S1 and H1 only (dL/df), the others written as zeros.
template <int Q, bool FULL>
__global__ void __launch_bounds__(kStage)
    k_bwd_nodes_split(PointRecs rec, const float4* __restrict__ rec32,
                      int64_t chunk, const double* __restrict__ tx,
                      const float4* __restrict__ s4, int64_t n_pad, double* __restrict__ part) {
  __shared__ float4 stage[2][kStage];
  const int64_t c = blockIdx.y;
  const int64_t k0 = (int64_t)blockIdx.x * kStage * Q + threadIdx.x;
  const int64_t p0 = c * chunk;
  const float4* p32 = rec32 + p0;
  float kh[Q], kl[Q], s1[Q], s2[Q], s3[Q], s4v[Q];
  double xk[Q], S1[Q], S2[Q], S3[Q], S4[Q], H1[Q], H2[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t k = k0 + (int64_t)q * kStage;
    const int64_t kc = k < n_pad ? k : n_pad - 1;
    const float4 nr = s4[kc];
    kh[q] = nr.x;
    kl[q] = nr.y;
    xk[q] = tx[kc];
    s1[q] = s2[q] = s3[q] = s4v[q] = 0.0f;
    S1[q] = S2[q] = S3[q] = S4[q] = H1[q] = H2[q] = 0.0;
  }

  staged_tiles(
      stage, p32, chunk,
      [&](const float4(&rc)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float t = (rc[i].x - kh[q]) + (rc[i].y - kl[q]);
            t = __builtin_amdgcn_rcpf(t);
            s1[q] = __builtin_fmaf(rc[i].z, t, s1[q]);
            if constexpr (FULL) {
              const float t2 = t * t;
              s2[q] = __builtin_fmaf(rc[i].w, t, s2[q]);
              s3[q] = __builtin_fmaf(rc[i].z, t2, s3[q]);
              s4v[q] = __builtin_fmaf(rc[i].w, t2, s4v[q]);
            }
          }
      },
      [&](int64_t b, int64_t end) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if (not_finite32(s1[q]) | not_finite32(s2[q]) | not_finite32(s3[q]) |
              not_finite32(s4v[q])) {
            for (int64_t p = b; p < end; ++p) {
              const int64_t pp = p0 + p;
              const float4 h = p32[p];
              const double pc = rec.c[pp], pcr = rec.cr[pp];
              if (h.x == h.x && rec.x[pp] != xk[q]) {
                // binary32 c: the binary32 reciprocal it was computed with
                if (pc == 0.0 && pcr == 0.0) continue;
                const double ti = (double)__builtin_amdgcn_rcpf((h.x - kh[q]) + (h.y - kl[q]));
                S1[q] = __builtin_fma(pc, ti, S1[q]);
                if (FULL) {
                  const double t2 = ti * ti;
                  S2[q] = __builtin_fma(pcr, ti, S2[q]);
                  S3[q] = __builtin_fma(pc, t2, S3[q]);
                  S4[q] = __builtin_fma(pcr, t2, S4[q]);
                }
              } else {
                bwd_pair_exact<FULL ? 2 : 1>(rec.x[pp], rec.c[pp], rec.cr[pp], rec.hg[pp],
                                             rec.hgr[pp], xk[q], S1[q], S2[q], S3[q], S4[q],
                                             H1[q], H2[q]);
              }
            }
          } else {
            S1[q] += (double)s1[q];
            S2[q] += (double)s2[q];
            S3[q] += (double)s3[q];
            S4[q] += (double)s4v[q];
          }
          s1[q] = s2[q] = s3[q] = s4v[q] = 0.0f;
        }
      });

  double* out = part + c * kPartFields * n_pad;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t k = k0 + (int64_t)q * kStage;
    if (k >= n_pad) continue;
    out[0 * n_pad + k] = S1[q];
    out[1 * n_pad + k] = S2[q];
    out[2 * n_pad + k] = S3[q];
    out[3 * n_pad + k] = S4[q];
    out[4 * n_pad + k] = H1[q];
    out[5 * n_pad + k] = H2[q];
  }
}

// ------------------------------------------------------------- launcher --
const void* bwd_nodes_split_kernel(int q) {
  return q == 2 ? reinterpret_cast<const void*>(k_bwd_nodes_split<2, true>)
                : reinterpret_cast<const void*>(k_bwd_nodes_split<1, true>);
}

template <int Q, bool FULL>
static void launch_nodes_split(const BackwardPlan& p, const NodeTable& t, const BackwardBufs& b,
                               hipStream_t s) {
  const dim3 g2((unsigned)((p.n_pad + kStage * Q - 1) / (kStage * Q)), (unsigned)p.chunks);
  k_bwd_nodes_split<Q, FULL><<<g2, kStage, 0, s>>>(b.rec, b.rec32, p.chunk, t.x, t.s, t.n_pad,
                                                   b.part);
}

hipError_t launch_backward_split_passes(const double* x, const double* g, int64_t n, int64_t m,
                                        const NodeTable& t, const BackwardBufs& b,
                                        const int32_t* scale_exp, double* dx, bool nodes_pass,
                                        bool full, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  constexpr int P = 1;
  const dim3 g1((unsigned)((p.m_pad + kStage * P - 1) / (kStage * P)));
  if (dx)
    k_bwd_points_split<P, false, true><<<g1, kStage, 0, s>>>(x, g, m, p.m_pad, t.s, t.n_pad, t.x,
                                                             t.w, t.f, n, scale_exp, dx, b.rec,
                                                             b.rec32, nullptr);
  else
    k_bwd_points_split<P, false, false><<<g1, kStage, 0, s>>>(x, g, m, p.m_pad, t.s, t.n_pad,
                                                              t.x, t.w, t.f, n, scale_exp, dx,
                                                              b.rec, b.rec32, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !nodes_pass) return e;
  if (p.q == 2)
    full ? launch_nodes_split<2, true>(p, t, b, s) : launch_nodes_split<2, false>(p, t, b, s);
  else
    full ? launch_nodes_split<1, true>(p, t, b, s) : launch_nodes_split<1, false>(p, t, b, s);
  return hipGetLastError();
}

hipError_t launch_forward_saved_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                      const int32_t* scale, const BackwardBufs& b, double* r,
                                      double* dr, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  if (b.saved32 == nullptr) return hipErrorInvalidValue;
  constexpr int P = 1;
  const dim3 g1((unsigned)((p.m_pad + kStage * P - 1) / (kStage * P)));
  k_bwd_points_split<P, false, true, true><<<g1, kStage, 0, s>>>(
      x, nullptr, m, p.m_pad, t.s, t.n_pad, t.x, t.w, t.f, n, scale, dr, b.saved, b.saved32, r);
  return hipGetLastError();
}

hipError_t launch_backward_saved_split(const double* g, int64_t m, const NodeTable& t,
                                       const BackwardBufs& b, bool full, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  if (b.saved32 == nullptr) return hipErrorInvalidValue;
  k_bwd_scale_records_split<<<dim3((unsigned)((p.m_pad + 255) / 256)), 256, 0, s>>>(
      b.saved, b.saved32, g, m, p.m_pad, b.rec, b.rec32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.q == 2)
    full ? launch_nodes_split<2, true>(p, t, b, s) : launch_nodes_split<2, false>(p, t, b, s);
  else
    full ? launch_nodes_split<1, true>(p, t, b, s) : launch_nodes_split<1, false>(p, t, b, s);
  return hipGetLastError();
}

hipError_t launch_eval_deriv_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                   const int32_t* scale, double* r, double* dr, hipStream_t s) {
  if (m == 0) return hipSuccess;
  constexpr int P = 1;
  const dim3 grid((unsigned)((m + kStage * P - 1) / (kStage * P)));
  k_bwd_points_split<P, true, true><<<grid, kStage, 0, s>>>(x, nullptr, m, m, t.s, t.n_pad, t.x,
                                                            t.w, t.f, n, scale, dr, PointRecs{},
                                                            nullptr, r);
  return hipGetLastError();
}

}  // namespace fhk
