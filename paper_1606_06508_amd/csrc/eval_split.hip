// Precision-split evaluation (gfx950): binary32 terms, binary64 data.
//
//  - Points and nodes enter as binary32 head/tail pairs (x = hi + lo to
//    about 2^-48 relative); the difference is formed as
//    (x_hi - k_hi) + (x_lo - k_lo).  When x and x_k are within a factor two
//    the head difference is exact (Sterbenz), so points that sit next to a
//    node still get an accurate difference; a plain binary32 difference
//    would round such points onto the node.
//  - t = 1/delta with v_rcp_f32 (within one ulp on gfx950, no refinement),
//    per difference (G = 1) or by simultaneous inversion of the four
//    differences of a node quad (G = 4: one v_rcp_f32 of their product and
//    nine multiplications, about six binary32 roundings per t; a product
//    that is not a normal number flags the lane).
//  - Weights w_k and weighted values w_k f_k are the binary64 ones scaled
//    by exact powers of two 2^-e and 2^-ef and rounded to binary32 (packing
//    kernel); r = 2^(ef - e) N / D and Lambda = L / |D| restore them exactly.
//  - Terms and per-tile partial sums (kTile nodes) are binary32; each tile's
//    partials are added into binary64 accumulators, so the binary32
//    rounding error grows with the tile length, not with n.
//  - The quotient r = N / D and Lambda = L / |D| are binary64.
// A lane whose tile sums are not finite (an exact hit gives t = inf, a NaN
// point gives NaN, extreme data may overflow binary32), whose point lies
// outside the binary32 domain (more than one node span outside the nodes;
// a table outside the domain carries NaN weights), or whose point is too
// ill-conditioned for binary32 terms (the Lebesgue sum, always accumulated,
// exceeds kSplitLambdaGuard |D|), recomputes its point in binary64 with the
// binary64 kernel's group reciprocals (eval_point_f64, groups of four), and
// from there the exact-hit branch or the per-pair division path where that
// flags.
//
// Issue rate.  On gfx950 binary32 add/sub/fmac issue at twice the binary64
// rate only in the 32-bit VOP2 encoding with VGPR operands; an SGPR operand
// or the VOP3 encoding (needed for abs modifiers) drops them to the binary64
// rate.  So the node records are staged by the block in LDS (double
// buffered, one tile of 256 records per step) and read back with
// wave-uniform ds_read_b128 (a broadcast into VGPRs), and |t| and |w| for
// the Lebesgue sum are taken with an integer and rather than an abs
// modifier.  Every per-pair operation except the reciprocal is then VOP2.
#include "fh_internal.h"
#include "pair_math.h"
#include "split_math.h"

// A table that the packing finds too ill-conditioned for binary32 terms
// (split_table_wide: a Lebesgue function above 2^12 at one of 64 sampled
// interval midpoints) is evaluated with binary64 terms at every point
// instead (status word 4).

namespace fhk {

// B: the sums are taken by node tiles (split_block_sums<..., B>) when the
// table's weights alternate in sign, which *alt says (written by the
// packing); D, hence r, is then the same with and without Lambda.
template <int P, int G, bool R, bool L, bool B>
__global__ void __launch_bounds__(kStage)
    k_eval_split(const double* __restrict__ x, int64_t m, const float4* __restrict__ s4,
                 int64_t n_pad, const double* __restrict__ tx, const double* __restrict__ tw,
                 const double* __restrict__ twf, const double* __restrict__ f, int64_t n,
                 const int32_t* __restrict__ scale,
                 const uint32_t* __restrict__ alt, double* __restrict__ r,
                 double* __restrict__ lam) {
  __shared__ float4 stage[2][kStage];
  const double x_first = tx[0], x_last = tx[n - 1];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kStage * P + tid;
  // 0x7fffffff in a VGPR, opaque to constant folding: the lane id ANDed with
  // a run-time zero (n_pad < 2^62)
  const uint32_t mask =
      0x7fffffffu ^ (__builtin_amdgcn_mbcnt_lo(~0u, 0u) & (uint32_t)(n_pad >> 62));
  double xp[P], N[P], D[P], A[P];
  float xh[P], xl[P];
  bool bad[P], dom[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * kStage;
    xp[j] = x[idx < m ? idx : m - 1];
    xh[j] = (float)xp[j];
    xl[j] = (float)(xp[j] - (double)xh[j]);
    N[j] = D[j] = A[j] = 0.0;
    dom[j] = !in_split_domain(xp[j], x_first, x_last);
    bad[j] = dom[j];
  }

  if (__builtin_amdgcn_readfirstlane(scale[3]) != 0) {
    // a table too ill-conditioned for binary32 terms (status word 4, written
    // by the packing): binary64 terms for every point, block-uniformly
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t idx = base + j * kStage;
      if (idx >= m) continue;
      PointRLF e = eval_point_f64<R, L>(xp[j], tx, tw, twf, n_pad);
      if (e.flagged) {
        const PointRL ex = eval_point_exact<R, L>(xp[j], tx, tw, f, n);
        e.r = ex.r;
        e.l = ex.l;
      }
      if (R) r[idx] = e.r;
      if (L) lam[idx] = e.l;
    }
    return;
  }

  // the Lebesgue sum is always accumulated: the conditioning guard needs it
  bool blocks = false;
  if constexpr (B) {
    blocks = __builtin_amdgcn_readfirstlane(*alt) != 0;
    if (blocks)
      split_block_sums<P, R, true, G, true>(stage, s4, n_pad, mask, xh, xl, N, D, A, bad);
  }
  if (!blocks) split_block_sums<P, R, true, G>(stage, s4, n_pad, mask, xh, xl, N, D, A, bad);
  const int shift = scale[1];

  // Three groups of points, in this order so that little stays live across
  // the slower paths: points whose binary32 terms pass the guard; points
  // for binary64 terms (outside the binary32 domain, or flagged by the
  // guard); points whose binary32 sums are not finite (an exact hit, a NaN
  // point, a difference too small for binary32) or that the binary64 sums
  // flag too, which take the exact branch at once (its binary search finds
  // a hit without a pass over the nodes).
  bool wide64[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * kStage;
    wide64[j] = dom[j];
    if (idx >= m || bad[j]) continue;
    double a = A[j];
    if constexpr (B)
      if (blocks) a = split_tile_fix<G>(xp[j], xh[j], xl[j], tx, n, s4, n_pad, mask, a);
    if (!(a <= kSplitLambdaGuard * fabs(D[j]))) {
      bad[j] = wide64[j] = true;
      continue;
    }
    if (R) r[idx] = ldexp(N[j] / D[j], shift);
    if (L) lam[idx] = a / fabs(D[j]);
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * kStage;
    if (idx >= m || !wide64[j]) continue;
    const PointRLF e = eval_point_f64<R, L>(xp[j], tx, tw, twf, n_pad);
    if (e.flagged) continue;
    bad[j] = false;
    if (R) r[idx] = e.r;
    if (L) lam[idx] = e.l;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * kStage;
    if (idx >= m || !bad[j]) continue;
    const PointRL ex = eval_point_exact<R, L>(xp[j], tx, tw, f, n);
    if (R) r[idx] = ex.r;
    if (L) lam[idx] = ex.l;
  }
}

template <int P, int G, bool B>
static hipError_t launch_v(const double* x, int64_t m, const NodeTable& t, int64_t n,
                           const int32_t* sc, const uint32_t* alt, double* r, double* lam,
                           hipStream_t s) {
  const int64_t per = (int64_t)kStage * P;
  const dim3 grid((unsigned)((m + per - 1) / per)), block(kStage);
  if (r && lam)
    k_eval_split<P, G, true, true, B><<<grid, block, 0, s>>>(x, m, t.s, t.n_pad, t.x, t.w, t.wf,
                                                             t.f, n, sc, alt, r, lam);
  else if (r)
    k_eval_split<P, G, true, false, B><<<grid, block, 0, s>>>(x, m, t.s, t.n_pad, t.x, t.w, t.wf,
                                                              t.f, n, sc, alt, r, lam);
  else
    k_eval_split<P, G, false, true, B><<<grid, block, 0, s>>>(x, m, t.s, t.n_pad, t.x, t.w, t.wf,
                                                              t.f, n, sc, alt, r, lam);
  return hipGetLastError();
}

// Variant table: id -> (points per lane P, reciprocal group G, sums by node
// tiles B); the node split is always 1 here (all waves of a block share the
// staged node tile).
#define FH_SPLIT_VARIANTS(X)                                                               \
  X(0, 1, 1, 0) X(1, 2, 1, 0) X(2, 4, 1, 0) X(3, 8, 1, 0) X(4, 1, 4, 0) X(5, 2, 4, 0)      \
  X(6, 4, 4, 0) X(7, 8, 4, 0) X(8, 1, 4, 1) X(9, 2, 4, 1) X(10, 4, 4, 1) X(11, 8, 4, 1)

int split_variant_count() {
#define FH_COUNT(id, p, g, b) +1
  return 0 FH_SPLIT_VARIANTS(FH_COUNT);
#undef FH_COUNT
}

void split_variant_shape(int id, int* p, int* g, int* s) {
  *s = 1;
  switch (id) {
#define FH_SHAPE(vid, vp, vg, vb) \
  case vid:                       \
    *p = vp;                      \
    *g = vg;                      \
    return;
    FH_SPLIT_VARIANTS(FH_SHAPE)
#undef FH_SHAPE
    default: *p = *g = 0;
  }
}

int split_variant_block(int id) {
  switch (id) {
#define FH_BLOCK(vid, vp, vg, vb) \
  case vid: return vb ? kTile : 0;
    FH_SPLIT_VARIANTS(FH_BLOCK)
#undef FH_BLOCK
    default: return 0;
  }
}

hipError_t launch_eval_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                             const int32_t* scale, const uint32_t* alt, double* r, double* lam,
                             const EvalConfig& cfg, hipStream_t s) {
  if (m == 0) return hipSuccess;
  switch (cfg.variant) {
#define FH_CASE(vid, vp, vg, vb) \
  case vid: return launch_v<vp, vg, vb != 0>(x, m, t, n, scale, alt, r, lam, s);
    FH_SPLIT_VARIANTS(FH_CASE)
#undef FH_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fhk
