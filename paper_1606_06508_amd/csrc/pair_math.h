// Binary64 pair arithmetic shared by the evaluation and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fhk {

// Node-pair records of the binary64 pair variants.  The node table is cut
// into blocks of kPairBlock records; block b holds the pairs (4i, 4i+2)
// ("even", i = 0..3) and (4i+1, 4i+3) ("odd") of its records in kPairRec
// doubles: {c, ok, lo, hi} (lo, hi: the nodes just before and after the
// block, -inf / +inf at the ends), then for the even and the odd pairs in
// turn the four m, the four -hh^2 and the four B, J, C and K
// (pack_pair_records).
constexpr int64_t kPairBlock = 16;
constexpr int64_t kPairHead = 4;
constexpr int64_t kPairRec = kPairHead + 48;

// true if v is +-0, subnormal, infinite or NaN (everything but normal)
__device__ __forceinline__ bool not_normal(double v) {
  return __builtin_amdgcn_class(v, 0x2F7);
}

// 1/q to about 2^-48.7 relative: the hardware estimate (at most 2^-24.37,
// measured) squared by one Newton step, plus its rounding
__device__ __forceinline__ double rcp_refined(double q) {
  const double y = __builtin_amdgcn_rcp(q);
  const double e = __builtin_fma(-q, y, 1.0);
  return __builtin_fma(y, e, y);
}

// Reciprocals of G deltas via one reciprocal of their product q, which is
// returned: if q is not a normal number the lane must be recomputed.
template <int G>
__device__ __forceinline__ double group_product_reciprocals(const double (&d)[G], double (&t)[G]);

template <>
__device__ __forceinline__ double group_product_reciprocals<4>(const double (&d)[4],
                                                              double (&t)[4]) {
  const double q01 = d[0] * d[1], q23 = d[2] * d[3];
  const double q = q01 * q23;
  const double y = rcp_refined(q);
  const double y01 = y * q23, y23 = y * q01;
  t[0] = y01 * d[1];
  t[1] = y01 * d[0];
  t[2] = y23 * d[3];
  t[3] = y23 * d[2];
  return q;
}

template <>
__device__ __forceinline__ double group_product_reciprocals<8>(const double (&d)[8],
                                                              double (&t)[8]) {
  const double q01 = d[0] * d[1], q23 = d[2] * d[3], q45 = d[4] * d[5], q67 = d[6] * d[7];
  const double q03 = q01 * q23, q47 = q45 * q67;
  const double q = q03 * q47;
  const double y = rcp_refined(q);
  const double y03 = y * q47, y47 = y * q03;
  const double y01 = y03 * q23, y23 = y03 * q01, y45 = y47 * q67, y67 = y47 * q45;
  t[0] = y01 * d[1];
  t[1] = y01 * d[0];
  t[2] = y23 * d[3];
  t[3] = y23 * d[2];
  t[4] = y45 * d[5];
  t[5] = y45 * d[4];
  t[6] = y67 * d[7];
  t[7] = y67 * d[6];
  return q;
}

// As group_product_reciprocals; returns true if the product is not normal.
template <int G>
__device__ __forceinline__ bool group_reciprocals(const double (&d)[G], double (&t)[G]) {
  return not_normal(group_product_reciprocals<G>(d, t));
}

// Index j with tx[j] == t among the strictly increasing tx[0, n), or -1
// (binary search; NaN never matches).
__device__ __forceinline__ int64_t find_node(double t, const double* __restrict__ tx, int64_t n) {
  int64_t lo = 0, hi = n - 1;
  if (t != t) return -1;
  while (lo <= hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    const double v = tx[mid];
    if (v == t) return mid;
    if (v < t)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// r and Lambda of one point, as eval_point_exact returns them (in registers:
// the out-of-line call then needs no private memory).
struct PointRL {
  double r, l;
};

// Exact per-pair evaluation of one point (flagged lanes only).  A NaN or
// infinite point gives NaN (every a_k is NaN or 0: r = Lambda = NaN); an
// exact hit is looked up by binary search (r = f_j, Lambda = 1); anything
// else -- products that leave the binary64 range -- takes one IEEE division
// per pair in a loop without early exits, so its loads pipeline (a flagged
// lane holds its whole wave).
template <bool R, bool L>
__device__ __noinline__ PointRL eval_point_exact(double t, const double* __restrict__ tx,
                                                 const double* __restrict__ tw,
                                                 const double* __restrict__ f, int64_t n) {
  if (!__builtin_isfinite(t)) return {__builtin_nan(""), __builtin_nan("")};
  const int64_t j = find_node(t, tx, n);
  if (j >= 0) return {R ? f[j] : 0.0, 1.0};
  double N = 0.0, D = 0.0, A = 0.0;
#pragma unroll 4
  for (int64_t k = 0; k < n; ++k) {
    const double del = t - tx[k];
    const double a = tw[k] / del;
    if (R) N = __builtin_fma(a, f[k], N);
    D = D + a;
    if (L) A = A + fabs(a);
  }
  return {N / D, A / fabs(D)};
}

// Fused sums of one wave over the node records [k_begin, k_end) (wave-
// uniform range, a multiple of G, below 2^31 records): for each of the
// lane's P points, D += w t, N += (w f) t, A += |w| |t|, with t from
// group_product_reciprocals<G>.  The loop counter is 32-bit, so loop control
// stays on the scalar unit.
//
// No range test inside the loop.  A group product q that is zero (an exact
// hit), infinite or NaN makes the refined reciprocal NaN (its Newton step
// forms 0 * inf or inf * 0), and so does a subnormal q whose estimate
// overflows; a NaN y makes every t of the group NaN and with it D, whatever
// the weights (w t is NaN even for w = 0).  One test of D per point after
// the loop therefore flags every lane that a test of each q would flag,
// except a subnormal q in (2^-1024, 2^-1022) whose reciprocal is finite: its
// terms stay correct to within 2^-51 of q's rounding instead of 2^-53.
template <int P, int G, bool R, bool L>
__device__ __forceinline__ void accumulate_f64(const double (&xp)[P], const double* __restrict__ tx,
                                               const double* __restrict__ tw,
                                               const double* __restrict__ twf, int64_t k_begin,
                                               int64_t k_end, double (&N)[P], double (&D)[P],
                                               double (&A)[P], bool (&bad)[P]) {
  const double* __restrict__ px = tx + k_begin;
  const double* __restrict__ pw = tw + k_begin;
  const double* __restrict__ pv = twf + k_begin;
  const int cnt = (int)(k_end - k_begin);
  for (int k = 0; k < cnt; k += G) {
    double xk[G], wk[G], vk[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      xk[i] = px[k + i];
      wk[i] = pw[k + i];
      vk[i] = R ? pv[k + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      double dl[G], t[G];
#pragma unroll
      for (int i = 0; i < G; ++i) dl[i] = xp[j] - xk[i];
      group_product_reciprocals<G>(dl, t);
#pragma unroll
      for (int i = 0; i < G; ++i) {
        D[j] = __builtin_fma(wk[i], t[i], D[j]);
        if (R) N[j] = __builtin_fma(vk[i], t[i], N[j]);
        if (L) A[j] = __builtin_fma(fabs(wk[i]), fabs(t[i]), A[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
}

// Number of nodes tx[0, n) below v (v finite; tx strictly increasing;
// n <= FH_MAX_NODES, so 32-bit indices: half the instructions of 64-bit
// ones on the vector unit).
__device__ __forceinline__ int64_t nodes_below(double v, const double* __restrict__ tx, int64_t n) {
  int32_t lo = 0, hi = (int32_t)n;
  while (lo < hi) {
    const int32_t mid = (int32_t)((uint32_t)(lo + hi) >> 1);
    if (tx[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Fused sums with the Lebesgue sum taken by blocks of U nodes, for weights
// that alternate in sign (Floater-Hormann weights do: every term of w_k has
// the sign (-1)^(k-d)).  On a block that lies on one side of the point all
// t_k share a sign, so |w_k t_k| alternates like w_k: the block's
// sum_k |w_k t_k| is |E - O| and its sum_k w_k t_k is E + O, with E and O
// the sums of w_k t_k over the block's even and odd records.  Each pair
// costs one multiply-add for both sums (two with the plain scheme), each
// block four additions.  Without L the block sums still form D, so r does
// not depend on whether Lambda is requested.  The one block that holds
// nodes on both sides of the point is wrong in A: the caller replaces its
// term afterwards (lebesgue_block_fix).  Lane flags as in accumulate_f64
// (D not finite).
template <int P, int G, int U, bool R, bool L>
__device__ __forceinline__ void accumulate_f64_blocks(const double (&xp)[P],
                                                      const double* __restrict__ tx,
                                                      const double* __restrict__ tw,
                                                      const double* __restrict__ twf,
                                                      int64_t k_begin, int64_t k_end,
                                                      double (&N)[P], double (&D)[P],
                                                      double (&A)[P], bool (&bad)[P]) {
  static_assert(U % G == 0, "blocks of whole node groups");
  const double* __restrict__ px = tx + k_begin;
  const double* __restrict__ pw = tw + k_begin;
  const double* __restrict__ pv = twf + k_begin;
  const int cnt = (int)(k_end - k_begin);
  for (int k = 0; k < cnt; k += U) {
    // E = sum of w_k t_k over the block's even records, O over its odd ones
    // (lebesgue_block_replace repeats these operations in this order)
    double E[P], O[P];
#pragma unroll
    for (int j = 0; j < P; ++j) E[j] = O[j] = 0.0;
    // one node group per iteration, as in accumulate_f64: unrolling the
    // block's groups lets the scheduler overlap them for all P points, at
    // several times the registers
#pragma unroll 1
    for (int h = 0; h < U; h += G) {
      double xk[G], wk[G], vk[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        xk[i] = px[k + h + i];
        wk[i] = pw[k + h + i];
        vk[i] = R ? pv[k + h + i] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < P; ++j) {
        double dl[G], t[G];
#pragma unroll
        for (int i = 0; i < G; ++i) dl[i] = xp[j] - xk[i];
        group_product_reciprocals<G>(dl, t);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (R) N[j] = __builtin_fma(vk[i], t[i], N[j]);
          if (i & 1)
            O[j] = __builtin_fma(wk[i], t[i], O[j]);
          else
            E[j] = __builtin_fma(wk[i], t[i], E[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      D[j] += E[j] + O[j];
      if (L) A[j] += fabs(E[j] - O[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
}

// The Lebesgue sum A of accumulate_f64_blocks with the term of the block
// at px/pw (U node records) replaced: A holds |E - O| for that block, which
// is right only if the block lies on one side of the point v; it gets
// sum_k |w_k t_k| instead, with E and O recomputed by the loop's operations
// (so the term removed is the term added).  (One refined reciprocal per
// pair instead of the group inversion needs fewer registers but more issue
// slots, and measured slower.)
template <int G, int U>
__device__ __forceinline__ double lebesgue_block_replace(double v, const double* __restrict__ px,
                                                         const double* __restrict__ pw,
                                                         double A) {
  double E = 0.0, O = 0.0, exact = 0.0;
  // one group at a time (once per point: few registers matter more here)
#pragma unroll 1
  for (int h = 0; h < U; h += G) {
    double dl[G], t[G];
#pragma unroll
    for (int i = 0; i < G; ++i) dl[i] = v - px[h + i];
    group_product_reciprocals<G>(dl, t);
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const double wk = pw[h + i];
      if (i & 1)
        O = __builtin_fma(wk, t[i], O);
      else
        E = __builtin_fma(wk, t[i], E);
      exact = __builtin_fma(fabs(wk), fabs(t[i]), exact);
    }
  }
  return (A - fabs(E - O)) + exact;
}

// A of accumulate_f64_blocks over the whole table, corrected: if the point v
// (finite, not a node) lies strictly inside block b (nodes x_{bU} ..
// x_{bU+U-1} on both sides of it, found by binary search), that block's
// term is replaced.  tx/tw are the padded tables (length a multiple of U),
// n the node count.
template <int G, int U>
__device__ __forceinline__ double lebesgue_block_fix(double v, const double* __restrict__ tx,
                                                     const double* __restrict__ tw, int64_t n,
                                                     double A) {
  const int64_t j = nodes_below(v, tx, n);
  if (j == 0 || j >= n || j % U == 0) return A;
  const int64_t b = j - j % U;
  return lebesgue_block_replace<G, U>(v, tx + b, tw + b, A);
}

// ---- Pair records (written by the packings) ----
//
// Block b holds records 16b .. 16b+15 (records at or beyond n repeat
// x_{n-1} with zero weight).  With the block's anchor c = (x_first +
// x_last) / 2 and, for each pair (a, a+2) of its even or odd records,
// a' = x_a - c, b' = x_{a+2} - c, m = (a' + b') / 2, hh = (b' - a') / 2,
//   B = w_a + w_{a+2},  J = (w_{a+2} - w_a) hh,
//   C = v_a + v_{a+2},  K = (v_{a+2} - v_a) hh      (v = w f as stored),
// the pair's two terms are, with x'' = (x - c) - m,
//   w_a / (x - x_a) + w_{a+2} / (x - x_{a+2}) = (B x'' + J) / (x''^2 - hh^2)
// and likewise (C x'' + K) / (x''^2 - hh^2) for v.  The header {c, ok, lo,
// hi} holds lo, hi = the nodes just before and after the block (-inf, +inf
// at the ends) and ok = 1 when every entry is finite and at most 2^480 in
// magnitude (so the products with x'' stay finite wherever x''^2 does) and
// the block is narrow next to the node spacings s_l, s_r just outside it:
// pair spans 2 hh at most kPairSpanMax and |a'|, |b'| at most
// kPairExtentMax times min(s_l, s_r).  A point outside the block and beyond
// those spacings is then at least min(s_l, s_r) from every node of the
// block, which bounds the first-order error of the pair terms there (see
// the accuracy note below).  A block with no node below n (only padding,
// zero weights) has ok = 1 as well.  The sums take a block with ok = 0 node
// by node (pair_block_nodes).  x: the table's n nodes; bw, bv: the block's 16
// weights and weighted values.  Contraction is off: the records do not
// depend on the compiler's choice of fused operations.
constexpr double kPairSpanMax = 8.0, kPairExtentMax = 16.0;

__device__ __forceinline__ double pair_anchor(const double* __restrict__ x, int64_t n,
                                              int64_t k0) {
#pragma clang fp contract(off)
  return 0.5 * (x[k0 < n ? k0 : n - 1] + x[k0 + 15 < n ? k0 + 15 : n - 1]);
}

__device__ __forceinline__ void pair_entries(const double* __restrict__ x, int64_t n, int64_t k0,
                                             double c, int a, const double* bw,
                                             const double* bv, double (&o)[6], double* ext,
                                             double* span) {
#pragma clang fp contract(off)
  const int64_t ka = k0 + a, kb = k0 + a + 2;
  const double ap = x[ka < n ? ka : n - 1] - c, bp = x[kb < n ? kb : n - 1] - c;
  const double m = 0.5 * (ap + bp), hh = 0.5 * (bp - ap);
  const double wa = bw[a], wb = bw[a + 2], va = bv[a], vb = bv[a + 2];
  o[0] = m;
  o[1] = -(hh * hh);
  o[2] = wa + wb;
  o[3] = (wb - wa) * hh;
  o[4] = va + vb;
  o[5] = (vb - va) * hh;
  *ext = fmax(fabs(ap), fabs(bp));
  *span = bp - ap;
}

// Pair t (0..7: even pairs 0..3, odd pairs 4..7) of the block at k0.
__device__ __forceinline__ void pair_record_pair(const double* __restrict__ x, int64_t n,
                                                 int64_t k0, const double* bw, const double* bv,
                                                 int t, double* __restrict__ rec) {
  const int g = t >> 2, i = t & 3;
  double o[6], ext, span;
  pair_entries(x, n, k0, pair_anchor(x, n, k0), 4 * i + g, bw, bv, o, &ext, &span);
#pragma unroll
  for (int f = 0; f < 6; ++f) rec[kPairHead + 24 * g + 4 * f + i] = o[f];
}

// The header of the block at k0; returns its ok (the block passed the test
// or holds no node).
__device__ __forceinline__ bool pair_record_header(const double* __restrict__ x, int64_t n,
                                                   int64_t k0, const double* bw,
                                                   const double* bv, double* __restrict__ rec) {
#pragma clang fp contract(off)
  const double c = pair_anchor(x, n, k0);
  bool ok = k0 < n && fabs(c) <= 0x1p480;
  double ext_max = 0.0, span_max = 0.0;
  for (int t = 0; t < 8; ++t) {
    double o[6], ext, span;
    pair_entries(x, n, k0, c, 4 * (t & 3) + (t >> 2), bw, bv, o, &ext, &span);
    for (int f = 0; f < 6; ++f) ok = ok && fabs(o[f]) <= 0x1p480;
    ext_max = fmax(ext_max, ext);
    span_max = fmax(span_max, span);
  }
  const double inf = __builtin_inf();
  const double sl = k0 >= 1 && k0 < n ? x[k0] - x[k0 - 1] : inf;
  const double sr = k0 + 16 < n ? x[k0 + 16] - x[k0 + 15] : inf;
  const double so = fmin(sl, sr);
  ok = (ok && so > 0.0 && so < inf && span_max <= kPairSpanMax * so &&
        ext_max <= kPairExtentMax * so) ||
       k0 >= n;
  rec[0] = c;
  rec[1] = ok ? 1.0 : 0.0;
  // the nodes just outside the block (lo < x <= hi: the block holds a node
  // next to x)
  rec[2] = k0 >= 1 && k0 <= n ? x[k0 - 1] : -inf;
  rec[3] = k0 + 16 < n ? x[k0 + 16] : inf;
  return ok;
}

// ---- Sums by node pairs ----
//
// Two records (a, a+2) of a block contribute, to D (B, J) or N (C, K),
//   w_a / (x - x_a) + w_{a+2} / (x - x_{a+2}) = (B x'' + J) / (x''^2 - hh^2),
// x'' = (x - c) - m (record layout and coefficients above).
// Per pair that is one subtraction, three multiply-adds, one reciprocal of
// a simultaneous inversion of four denominators and one multiply-add per
// sum: 9 issue slots for two (point, node) pairs with both sums against 12
// node by node.  The even pairs of a block form E, its odd pairs O, so the
// block's Lebesgue term is |E - O| as in accumulate_f64_blocks.
//
// Accuracy.  The pair form evaluates (d_a, d_b) = x'' +- hh through x - c
// and the rounded m, hh, and its numerators through the monomials B x'' and
// J, so its error is relative to distances of the block's size: at a point
// at distance delta >= s from the block (s the smaller node spacing just
// outside it, spans 2 hh <= rho s and |a'|, |b'| <= sigma s by the pack's
// test), each pair term w_a / d_a + w_b / d_b is perturbed relatively by at
// most about (2 + 4 sigma + rho / 2) u through the differences,
// (1 + rho / 4) u through the denominator x''^2 - hh^2, (2 + 3 rho / 2) u
// through the numerator, and the reciprocal's 27 u: (32 + 4 sigma + 9 rho / 4) u,
// at most 114 u with sigma <= 16, rho <= 8 (a few u for blocks further away).
// Closer to the block, the terms have no such bound, so the blocks of the
// point's two neighbouring nodes x_{j-1} < x <= x_j (one block, or two when
// the point lies between blocks) are masked out of the loop and summed node
// by node afterwards (pair_fix_point): every other block is then at least
// one outer spacing away from the point.  Block b holds node j-1 or j
// exactly when lo_b < x <= hi_b, lo_b and hi_b the nodes just before and
// after it: two compares with scalar operands per block and point, no
// search.
//
// Masking multiplies the block's sums by 0 or 1, so a non-finite value in a
// masked block (a hit, or a denominator that cancels to zero) still makes D
// NaN and sends the lane to eval_point_exact; finite garbage vanishes.

// One pair group (four pairs; entries at g: m[4], -hh^2[4], B, J, C, K) at
// the P points x1 = x - c: S = sum (B x'' + J) / q, Nb (+)= sum (C x'' + K) / q;
// first_n: Nb starts at the group's terms.  JKL: the group's J[4], K[4]
// come from jk (LDS, staged by pair_stage_jk), read into VGPRs by the LDS
// pipe.
template <int P, bool R, bool JKL>
__device__ __forceinline__ void pair_group(const double (&x1)[P], const double* __restrict__ g,
                                           const double* jk, double (&Nb)[P], double (&S)[P],
                                           bool first_n) {
  double pm[4], pq[4], pB[4], pJ[4], pC[4], pK[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    pm[i] = g[i];
    pq[i] = g[4 + i];
    pB[i] = g[8 + i];
    pJ[i] = JKL ? jk[i] : g[12 + i];
    pC[i] = R ? g[16 + i] : 0.0;
    pK[i] = R ? (JKL ? jk[4 + i] : g[20 + i]) : 0.0;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    double q[4], nd[4], nn[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double xx = x1[j] - pm[i];
      q[i] = __builtin_fma(xx, xx, pq[i]);
      nd[i] = __builtin_fma(pB[i], xx, pJ[i]);
      if (R) nn[i] = __builtin_fma(pC[i], xx, pK[i]);
    }
    group_product_reciprocals<4>(q, y);
    S[j] = nd[0] * y[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) S[j] = __builtin_fma(nd[i], y[i], S[j]);
    if (R) {
      Nb[j] = first_n ? nn[0] * y[0] : __builtin_fma(nn[0], y[0], Nb[j]);
#pragma unroll
      for (int i = 1; i < 4; ++i) Nb[j] = __builtin_fma(nn[i], y[i], Nb[j]);
    }
  }
}

// ---- Octets: node blocks far from the points ----
//
// The even records of a 16-node block (0, 2, ..., 14), and likewise its odd
// ones, have weights of one sign, and their eight terms add up to one
// rational function of the octet's coordinate y = (x - c) - m (c the block's
// anchor, m the midpoint of the octet's first and last offset a' = x_k - c,
// r_i = a'_i - m its roots):
//   sum_i w_i / (y - r_i) = PD(y) / Q(y),   Q(y) = prod_i (y - r_i),
//   PD(y) = sum_i w_i prod_{j != i} (y - r_j),
// and likewise PN with the weighted values v_i.  Q is monic of degree 8,
// PD and PN of degree 7, all evaluated from their monomial coefficients by
// Horner's rule: one subtraction and 8 + 7 (+ 7) operations for eight
// nodes, and one reciprocal for the block's two octets.  Horner's rule errs
// by at most about k u sum_k |c_k| |y|^k, and the coefficients as
// multiplied out carry errors of the same form; relative to the sum of
// |w_i / (y - r_i)| both amount to about (8 + 8 + 7 + 7) u times
// F(y) = prod_i (|y| + |r_i|) / |y - r_i|, which falls as |y| grows.  A block
// takes octets only for points with at least kOctetGap whole blocks between
// it and the blocks of the points' neighbouring nodes, so the closest
// points it serves are the nodes x_{16b - 16 kOctetGap - 1} and
// x_{16b + 16 (kOctetGap + 1)}; an octet passes when F there is at most
// kOctetFactorMax (equispaced nodes: F <= 2.24, Chebyshev nodes <= 5.7)
// and its coordinates (|y| <= 2^50, distances >= 2^-50) and coefficients
// (<= 2^400) keep every intermediate a normal number.
constexpr int kOctetGap = 2;
constexpr double kOctetFactorMax = 8.0;

// coefficients t[0..deg] times (y - r), in place (t has room for deg + 2)
__device__ __forceinline__ void octet_times_root(double* t, int deg, double r) {
  t[deg + 1] = t[deg];
  for (int k = deg; k >= 1; --k) t[k] = __builtin_fma(-r, t[k], t[k - 1]);
  t[0] = -r * t[0];
}

// Octet g (0: even, 1: odd records) of the block at k0 with anchor c (x,
// w, v: the table's n nodes, weights and weighted values; records at or
// beyond n repeat x_{n-1} with zero weight): o[0] = m, o[1..8] = Q[0..7]
// (Q = y^8 + sum_k Q[k] y^k), o[9..16] = PD[0..7] and, with V,
// o[17..24] = PN[0..7]; returns whether it passed.
template <bool V>
__device__ bool octet_coefficients(const double* __restrict__ x, const double* __restrict__ w,
                                   const double* __restrict__ v, int64_t n, int64_t k0, double c,
                                   int g, double* __restrict__ o) {
#pragma clang fp contract(off)
  double a[8], wi[8], vi[8], r[8];
  for (int i = 0; i < 8; ++i) {
    const int64_t k = k0 + g + 2 * i;
    a[i] = x[k < n ? k : n - 1] - c;
    wi[i] = k < n ? w[k] : 0.0;
    vi[i] = V && k < n ? v[k] : 0.0;
  }
  const double m = 0.5 * (a[0] + a[7]);
  double rho = 0.0;
  for (int i = 0; i < 8; ++i) {
    r[i] = a[i] - m;
    rho = fmax(rho, fabs(r[i]));
  }
  double q[9] = {1.0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 8; ++i) octet_times_root(q, i, r[i]);
  double pd[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pn[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 8; ++i) {
    double t[8] = {1.0, 0, 0, 0, 0, 0, 0, 0};
    int deg = 0;
    for (int j = 0; j < 8; ++j)
      if (j != i) octet_times_root(t, deg++, r[j]);
    for (int k = 0; k < 8; ++k) {
      pd[k] = __builtin_fma(wi[i], t[k], pd[k]);
      if (V) pn[k] = __builtin_fma(vi[i], t[k], pn[k]);
    }
  }
  bool ok = true;
  o[0] = m;
  for (int k = 0; k < 8; ++k) {
    o[1 + k] = q[k];
    o[9 + k] = pd[k];
    if (V) o[17 + k] = pn[k];
    ok = ok && fabs(q[k]) <= 0x1p400 && fabs(pd[k]) <= 0x1p400 && fabs(pn[k]) <= 0x1p400;
  }
  // the points the octet serves lie beyond the two closest ones
  const int64_t side[2] = {k0 - 16 * kOctetGap - 1, k0 + 16 * (kOctetGap + 1)};
  for (int e = 0; e < 2; ++e) {
    if (side[e] < 0 || side[e] > n - 1) continue;
    const double y = (x[side[e]] - c) - m;
    double f = 1.0, near = __builtin_inf();
    for (int i = 0; i < 8; ++i) {
      const double dy = fabs(y - r[i]);
      f *= (fabs(y) + fabs(r[i])) / dy;
      near = fmin(near, dy);
    }
    ok = ok && f <= kOctetFactorMax && near >= 0x1p-50;
  }
  const double far = fmax(fabs((x[0] - c) - m), fabs((x[n - 1] - c) - m));
  return ok && far + rho <= 0x1p50;
}

// Q and PD (and with V, PN) of one octet (o as written above) at y
template <bool V>
__device__ __forceinline__ void octet_eval(const double* __restrict__ o, double y, double& Q,
                                           double& PD, double& PN) {
  Q = y + o[8];
  for (int k = 7; k >= 1; --k) Q = __builtin_fma(Q, y, o[k]);
  PD = __builtin_fma(o[16], y, o[15]);
  for (int k = 14; k >= 9; --k) PD = __builtin_fma(PD, y, o[k]);
  if (V) {
    PN = __builtin_fma(o[24], y, o[23]);
    for (int k = 22; k >= 17; --k) PN = __builtin_fma(PN, y, o[k]);
  }
}

// Octet records of the evaluation: per block c, then the even and the odd
// octet with both numerators (25 doubles each), then the closest points the
// octets serve on either side, L = x_{16b - 16 kOctetGap - 1} and
// R = x_{16b + 16 (kOctetGap + 1)} (-inf / +inf where there is no such
// node: no point is served on that side), one spare.  A point x takes the
// block's octets exactly when x <= L or x >= R.
constexpr int64_t kOctetEvalRec = 54;

// A wave-uniform double as a scalar value (the same in every lane)
__device__ __forceinline__ double uniform_f64(double v) {
  const int64_t b = __builtin_bit_cast(int64_t, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((int64_t)hi << 32) | (int64_t)(uint32_t)lo);
}

// One block's sums from its two octets' values at a point: E = PDe / Qe,
// O = PDo / Qo (one reciprocal of Qe Qo) and Nb = PNe / Qe + PNo / Qo.  No
// contraction: every caller gets the same bits.
template <bool R>
__device__ __forceinline__ void octet_combine(double Qe, double PDe, double PNe, double Qo,
                                              double PDo, double PNo, double& Nb, double& E,
                                              double& O) {
#pragma clang fp contract(off)
  const double y = rcp_refined(Qe * Qo);
  const double te = y * Qo, to = y * Qe;
  E = PDe * te;
  O = PDo * to;
  if (R) Nb = __builtin_fma(PNe, te, PNo * to);
}

// What a wave knows of the octets (wave-uniform): the table's octet
// records, whether every block passed the octet test, and the smallest and
// largest of the wave's points.  Block b serves the points at or beyond its
// record's L and R; the launch sorts the points by the block of their
// neighbouring nodes, so that most blocks serve every point of a wave.
struct OctetView {
  const double* rec;
  bool on;
  double xmin, xmax;
  // (the compares run on the vector unit; readfirstlane makes the result a
  // scalar the branch can take)
  __device__ __forceinline__ bool far_for_all(const double* __restrict__ o) const {
    return __builtin_amdgcn_readfirstlane((int)(xmax <= o[51] || xmin >= o[52])) != 0;
  }
  __device__ __forceinline__ bool far_for_some(const double* __restrict__ o) const {
    return __builtin_amdgcn_readfirstlane((int)(xmin <= o[51] || xmax >= o[52])) != 0;
  }
};

// Whether the block's record passed the pack's test: the high word of its
// flag (1.0 or 0.0), an integer the scalar unit can branch on.
__device__ __forceinline__ bool pair_block_passed(const double* __restrict__ rec) {
  return __double2hiint(rec[1]) != 0;
}

// The sums of a block that failed the pack's test, node by node from the
// node table (px, pw, pv: the block's 16 records) in two groups of 8: the
// same quantities as the pair groups give, Nb = sum v_k t_k and E, O the
// sums of w_k t_k over the block's even and odd records.
template <int P, bool R>
__device__ __forceinline__ void pair_block_nodes(const double (&xp)[P],
                                                 const double* __restrict__ px,
                                                 const double* __restrict__ pw,
                                                 const double* __restrict__ pv, double (&Nb)[P],
                                                 double (&E)[P], double (&O)[P]) {
  constexpr int G = 8;
#pragma unroll
  for (int j = 0; j < P; ++j) Nb[j] = E[j] = O[j] = 0.0;
#pragma unroll 1
  for (int h = 0; h < (int)kPairBlock; h += G) {
    double xk[G], wk[G], vk[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      xk[i] = px[h + i];
      wk[i] = pw[h + i];
      vk[i] = R ? pv[h + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      double dl[G], t[G];
#pragma unroll
      for (int i = 0; i < G; ++i) dl[i] = xp[j] - xk[i];
      group_product_reciprocals<G>(dl, t);
#pragma unroll
      for (int i = 0; i < G; ++i) {
        if (R) Nb[j] = __builtin_fma(vk[i], t[i], Nb[j]);
        if (i & 1)
          O[j] = __builtin_fma(wk[i], t[i], O[j]);
        else
          E[j] = __builtin_fma(wk[i], t[i], E[j]);
      }
    }
  }
}

// Fused sums by node pairs over the records [k_begin, k_end) (wave-uniform,
// multiples of kPairBlock): for each block its pair sums, then N += Nb,
// D += E + O, A += |E - O|, each times 0 where the block holds a node next
// to the point (lo_b < x <= hi_b); the last such block is kept in rlast
// (untouched if none).  MIXED: some block of the table failed the pack's
// test; each block then checks its flag (wave-uniform, a scalar branch) and
// a failing one takes its sums node by node from the node table tx, tw, twf
// (pair_block_nodes), masked alike.  Without MIXED every block passed and
// the loop holds no such test.  Lane flags as in accumulate_f64 (D not
// finite).
//
// A VOP3 instruction reads at most one SGPR, so B x'' + J and C x'' + K
// cannot take both coefficients from the scalar unit.  With JKL (the
// table's J and K staged in jk_lds by pair_stage_jk) they come from LDS
// broadcast reads, which use the LDS pipe; without it they are copied from
// SGPRs to VGPRs, 16 moves per block shared by the lane's P points (vector
// loads from memory instead left their latency exposed, measured slower).
template <int P, bool R, bool L, bool JKL, bool MIXED, bool OCT = false>
__device__ __forceinline__ void accumulate_f64_pairs(
    const double (&xp)[P], const double* __restrict__ pr, const double* jk_lds,
    const double* __restrict__ tx, const double* __restrict__ tw, const double* __restrict__ twf,
    int64_t k_begin, int64_t k_end, double (&N)[P], double (&D)[P], double (&A)[P],
    bool (&bad)[P], int32_t (&rlast)[P], const OctetView* ov = nullptr) {
  const int b0 = (int)(k_begin / kPairBlock);
  const int nb = (int)((k_end - k_begin) / kPairBlock);
  for (int ib = 0; ib < nb; ++ib) {
    const int b = b0 + ib;
    if constexpr (OCT) {
      const double* __restrict__ o = ov->rec + (int64_t)b * kOctetEvalRec;
      if (ov->on && ov->far_for_all(o)) {
        // the block serves every point of the wave: its octets, no mask
        double x1[P], Qe[P], PDe[P], PNe[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          x1[j] = xp[j] - o[0];
          octet_eval<R>(o + 1, x1[j] - o[1], Qe[j], PDe[j], PNe[j]);
        }
        // the odd octet's coefficients load into the SGPRs of the even one's
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < P; ++j) {
          double Qo, PDo, PNo, Nb, E, O;
          octet_eval<R>(o + 26, x1[j] - o[26], Qo, PDo, PNo);
          octet_combine<R>(Qe[j], PDe[j], PNe[j], Qo, PDo, PNo, Nb, E, O);
          if (R) N[j] += Nb;
          D[j] += E + O;
          if (L) A[j] += fabs(E - O);
        }
        continue;
      }
    }
    const double* __restrict__ rec = pr + (int64_t)b * kPairRec;
    double Nb[P], E[P], O[P];
    const double lo_b = rec[2], hi_b = rec[3];
    if (!MIXED || pair_block_passed(rec)) {
      const double c = rec[0];
      double x1[P];
#pragma unroll
      for (int j = 0; j < P; ++j) x1[j] = xp[j] - c;
      const double* jk = jk_lds + b * (int)kPairBlock;
      pair_group<P, R, JKL>(x1, rec + kPairHead, jk, Nb, E, true);
      // the odd group's entries load into the SGPRs of the even group's
      // (48 SGPRs each)
      __builtin_amdgcn_sched_barrier(0);
      pair_group<P, R, JKL>(x1, rec + kPairHead + 24, jk + 8, Nb, O, false);
    } else {
      const int64_t k0 = (int64_t)b * kPairBlock;
      pair_block_nodes<P, R>(xp, tx + k0, tw + k0, twf + k0, Nb, E, O);
    }
    if constexpr (OCT) {
      const double* __restrict__ o = ov->rec + (int64_t)b * kOctetEvalRec;
      if (ov->on && ov->far_for_some(o)) {
        // the points the block serves take its octets (never masked: the
        // block holds neither of their neighbouring nodes)
        const double lo_o = o[51], hi_o = o[52];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!(xp[j] <= lo_o || xp[j] >= hi_o)) continue;
          const double x1 = xp[j] - o[0];
          double Qe, PDe, PNe, Qo, PDo, PNo;
          octet_eval<R>(o + 1, x1 - o[1], Qe, PDe, PNe);
          octet_eval<R>(o + 26, x1 - o[26], Qo, PDo, PNo);
          octet_combine<R>(Qe, PDe, PNe, Qo, PDo, PNo, Nb[j], E[j], O[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const bool near = xp[j] > lo_b && xp[j] <= hi_b;
      const double f = near ? 0.0 : 1.0;
      rlast[j] = near ? b : rlast[j];
      if (R) N[j] = __builtin_fma(f, Nb[j], N[j]);
      D[j] = __builtin_fma(f, E[j] + O[j], D[j]);
      if (L) A[j] = __builtin_fma(f, fabs(E[j] - O[j]), A[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
}

// Largest node range whose J and K the pair variants stage in LDS (8 B per
// record: 32 KB).
constexpr int64_t kPairLdsRecords = 4096;

// Copies J and K of the blocks [0, n_loop / 16) from the pair records into
// jk_lds ([block][J even[4], K even[4], J odd[4], K odd[4]]), all threads of
// the block taking part; the caller synchronizes.
__device__ __forceinline__ void pair_stage_jk(const double* __restrict__ pr, int64_t n_loop,
                                              double* jk_lds) {
  const int chunks = (int)(n_loop / kPairBlock) * 4;
  for (int i = threadIdx.x; i < chunks; i += blockDim.x) {
    const int b = i >> 2, g = (i >> 1) & 1, k = i & 1;
    const double* src = pr + (int64_t)b * kPairRec + kPairHead + 24 * g + (k ? 20 : 12);
    double* dst = jk_lds + b * kPairBlock + 8 * g + 4 * k;
    const double2 a = reinterpret_cast<const double2*>(src)[0];
    const double2 c = reinterpret_cast<const double2*>(src)[1];
    reinterpret_cast<double2*>(dst)[0] = a;
    reinterpret_cast<double2*>(dst)[1] = c;
  }
}

// True when every block of the records [0, n_loop) passed the pack's test
// (the pack's summary words: bit i of word w for block 16 w + i).
__device__ __forceinline__ bool pair_table_ok(const uint32_t* __restrict__ pok, int64_t n_loop) {
  const int64_t words = (n_loop / kPairBlock + 15) / 16;
  uint32_t all = 0xFFFFu;
  for (int64_t i = 0; i < words; ++i) all &= pok[i];
  return __builtin_amdgcn_readfirstlane(all) == 0xFFFFu;
}

// The masked blocks of accumulate_f64_pairs at the point v (not flagged),
// node by node: block rlast, and block rlast - 1 too when v is at or below
// the first node of block rlast (v then lies between the two blocks);
// N += v_k t, D += w_k t, A += |w_k| |t| with t from groups of G
// differences.  The loads take 32-bit byte offsets from the table bases,
// so one offset per group serves all of its loads.
template <int G, bool R, bool L>
__device__ __forceinline__ void pair_fix_point(double v, int32_t rlast,
                                               const double* __restrict__ tx,
                                               const double* __restrict__ tw,
                                               const double* __restrict__ twf, double& N,
                                               double& D, double& A) {
  const char* __restrict__ bx = reinterpret_cast<const char*>(tx);
  const char* __restrict__ bw = reinterpret_cast<const char*>(tw);
  const char* __restrict__ bv = reinterpret_cast<const char*>(twf);
  const uint32_t first = (uint32_t)rlast * (uint32_t)kPairBlock;
  const bool two = rlast > 0 && v <= tx[first];
#pragma unroll 1
  for (int32_t b = rlast - (two ? 1 : 0); b <= rlast; ++b) {
#pragma unroll 1
    for (int h = 0; h < (int)kPairBlock; h += G) {
      const uint32_t off = ((uint32_t)b * (uint32_t)kPairBlock + (uint32_t)h) * 8u;
      double dl[G], t[G], wk[G], vk[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        dl[i] = v - *reinterpret_cast<const double*>(bx + off + 8 * i);
        wk[i] = *reinterpret_cast<const double*>(bw + off + 8 * i);
        vk[i] = R ? *reinterpret_cast<const double*>(bv + off + 8 * i) : 0.0;
      }
      group_product_reciprocals<G>(dl, t);
#pragma unroll
      for (int i = 0; i < G; ++i) {
        if (R) N = __builtin_fma(vk[i], t[i], N);
        D = __builtin_fma(wk[i], t[i], D);
        if (L) A = __builtin_fma(fabs(wk[i]), fabs(t[i]), A);
      }
    }
  }
}

}  // namespace fhk
