// Precision-split evaluation (gfx950): binary32 terms, binary64 data.
//
//  - Points and nodes enter as binary32 head/tail pairs (x = hi + lo to
//    about 2^-48 relative); the difference is formed as
//    (x_hi - k_hi) + (x_lo - k_lo).  When x and x_k are within a factor two
//    the head difference is exact (Sterbenz), so points that sit next to a
//    node still get an accurate difference; a plain binary32 difference
//    would round such points onto the node.
//  - t = 1/delta with v_rcp_f32 (within one ulp on gfx950, no refinement).
//  - Weights are the binary64 weights scaled by an exact power of two and
//    rounded to binary32 (packing kernel); the scale cancels in r and
//    Lambda.
//  - Terms and per-tile partial sums (kTile nodes) are binary32; each tile's
//    partials are added into binary64 accumulators, so the binary32
//    rounding error grows with the tile length, not with n.
//  - The quotient r = N / D and Lambda = L / |D| are binary64.
// A lane whose tile sums are not finite (an exact hit gives t = inf, a NaN
// point gives NaN, extreme data may overflow binary32) recomputes its point
// with the binary64 per-pair division path and the exact-hit branch.
#include "fh_internal.h"

namespace fhk {

constexpr int kTile = 32;

__device__ __forceinline__ bool not_finite32(float v) {
  return __builtin_amdgcn_classf(v, 0x207);  // NaN or +-inf
}

template <bool R, bool L>
__device__ __noinline__ void eval_point_exact_s(double t, const double* __restrict__ tx,
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
    k_eval_split(const double* __restrict__ x, int64_t m, const float* __restrict__ sxh,
                 const float* __restrict__ sxl, const float* __restrict__ sw,
                 const float* __restrict__ swf, int64_t n_pad, const double* __restrict__ tx,
                 const double* __restrict__ tw, const double* __restrict__ f, int64_t n,
                 double* __restrict__ r, double* __restrict__ lam) {
  const int64_t stride = blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * stride * P + threadIdx.x;
  double xp[P], N[P], D[P], A[P];
  float xh[P], xl[P];
  bool bad[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * stride;
    xp[j] = x[idx < m ? idx : m - 1];
    xh[j] = (float)xp[j];
    xl[j] = (float)(xp[j] - (double)xh[j]);
    N[j] = 0.0;
    D[j] = 0.0;
    A[j] = 0.0;
    bad[j] = false;
  }

  for (int64_t k0 = 0; k0 < n_pad; k0 += kTile) {
    float Nt[P], Dt[P], At[P];
#pragma unroll
    for (int j = 0; j < P; ++j) Nt[j] = Dt[j] = At[j] = 0.0f;
#pragma unroll 8
    for (int kk = 0; kk < kTile; ++kk) {
      const int64_t k = k0 + kk;
      const float kh = sxh[k], kl = sxl[k], w = sw[k];
      const float v = R ? swf[k] : 0.0f;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const float del = (xh[j] - kh) + (xl[j] - kl);
        const float t = __builtin_amdgcn_rcpf(del);
        Dt[j] = __builtin_fmaf(w, t, Dt[j]);
        if (R) Nt[j] = __builtin_fmaf(v, t, Nt[j]);
        if (L) At[j] = __builtin_fmaf(fabsf(w), fabsf(t), At[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      bad[j] |= not_finite32(Dt[j]);
      D[j] += (double)Dt[j];
      if (R) {
        bad[j] |= not_finite32(Nt[j]);
        N[j] += (double)Nt[j];
      }
      if (L) {
        bad[j] |= not_finite32(At[j]);
        A[j] += (double)At[j];
      }
    }
  }

#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * stride;
    if (idx >= m) continue;
    double rv, lv;
    if (bad[j]) {
      eval_point_exact_s<R, L>(xp[j], tx, tw, f, n, &rv, &lv);
    } else {
      rv = N[j] / D[j];
      lv = A[j] / fabs(D[j]);
    }
    if (R) r[idx] = rv;
    if (L) lam[idx] = lv;
  }
}

template <int P>
static hipError_t launch_sp(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                            double* lam, int block, hipStream_t s) {
  const int64_t per = (int64_t)block * P;
  const dim3 grid((unsigned)((m + per - 1) / per));
  if (r && lam)
    k_eval_split<P, true, true><<<grid, block, 0, s>>>(x, m, t.sx_hi, t.sx_lo, t.sw, t.swf,
                                                       t.n_pad, t.x, t.w, t.f, n, r, lam);
  else if (r)
    k_eval_split<P, true, false><<<grid, block, 0, s>>>(x, m, t.sx_hi, t.sx_lo, t.sw, t.swf,
                                                        t.n_pad, t.x, t.w, t.f, n, r, lam);
  else
    k_eval_split<P, false, true><<<grid, block, 0, s>>>(x, m, t.sx_hi, t.sx_lo, t.sw, t.swf,
                                                        t.n_pad, t.x, t.w, t.f, n, r, lam);
  return hipGetLastError();
}

hipError_t launch_eval_split(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                             double* lam, const EvalConfig& cfg, hipStream_t s) {
  if (m == 0) return hipSuccess;
  switch (cfg.points_per_lane) {
    case 1: return launch_sp<1>(x, m, t, n, r, lam, cfg.block, s);
    case 2: return launch_sp<2>(x, m, t, n, r, lam, cfg.block, s);
    default: return launch_sp<4>(x, m, t, n, r, lam, cfg.block, s);
  }
}

}  // namespace fhk
