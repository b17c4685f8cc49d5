// Binary32 pair arithmetic of the precision-split kernels (single and
// batched): the LDS-staged node loop of one block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pair_math.h"

namespace fhk {

constexpr int kTile = 32;     // binary32 partial-sum length (nodes)
constexpr int kStage = 256;   // records per LDS stage (= threads per block)
// Conditioning guard of the split kernels: a point whose binary32-term
// Lebesgue function L / |D| exceeds this is recomputed in binary64.  The
// binary32 sums give |D^ - D| <= c u32 L with c <= 41 (first order), so an
// unflagged point has a true Lebesgue constant below about 2^16 (where
// c u32 Lambda <= 0.16 and the first-order split bound holds with a factor
// of at most 1.2), and a flagged one gets binary64 accuracy.
constexpr double kSplitLambdaGuard = 0x1p14;

// A pointer argument made provably wave-uniform (it is the same in every
// lane), so loads through it become scalar loads.
template <class T>
__device__ __forceinline__ const T* uniform_ptr(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// Binary64 evaluation of one point over a packed table (records [0, n_pad),
// n_pad a multiple of 4): the fused sums with groups of four differences per
// reciprocal and plain sums, the per-pair operations of the binary64 kernel
// with groups of four, no node split and plain sums (so the same bits;
// groups of eight would keep the split kernel from fitting eight waves per
// SIMD).  For the points of the split kernels whose binary32 terms cannot
// be trusted: all points of a table too ill-conditioned for them, and lanes
// that their per-point guard flags.  Inline, so that it shares the
// registers of the binary32 loop that ran before it (an out-of-line call
// adds its registers to the kernel's); the table is the same for every
// lane, so its records arrive through scalar loads.  `flagged` is set where
// the binary64 sums flag too (an exact hit, a NaN or infinite point, a group
// product out of range): the caller then takes eval_point_exact.
struct PointRLF {
  double r, l;
  bool flagged;
};

template <bool R, bool L>
__device__ __forceinline__ PointRLF eval_point_f64(double v, const double* __restrict__ tx,
                                                   const double* __restrict__ tw,
                                                   const double* __restrict__ twf,
                                                   int64_t n_pad) {
  tx = uniform_ptr(tx);
  tw = uniform_ptr(tw);
  twf = uniform_ptr(twf);
  n_pad = __builtin_amdgcn_readfirstlane((int32_t)n_pad);  // n_pad < 2^31
  double xp[1] = {v}, N[1] = {0.0}, D[1] = {0.0}, A[1] = {0.0};
  bool bad[1] = {false};
  accumulate_f64<1, 4, R, L>(xp, tx, tw, twf, 0, n_pad, N, D, A, bad);
  return {N[0] / D[0], A[0] / fabs(D[0]), bad[0]};
}

__device__ __forceinline__ bool not_finite32(float v) {
  return __builtin_amdgcn_classf(v, 0x207);  // NaN or +-inf
}

// |v| by clearing the sign bit with a VOP2 v_and_b32 against a mask held in
// a VGPR (an abs modifier, or an and with a known constant that the compiler
// folds into one, would force the slower VOP3 encoding).
__device__ __forceinline__ float abs_vop2(float v, uint32_t mask) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & mask);
}

// Reciprocals of four binary32 differences d[0..3] in place by simultaneous
// inversion: one v_rcp_f32 of the product q = (d0 d1)(d2 d3), then
// 1/d0 = y q23 d1 and so on (y ~ 1/q).  Nine multiplications and one
// quarter-rate reciprocal replace four reciprocals; each result carries
// about six binary32 roundings (three for q, the reciprocal's ulp, two on
// the way back) instead of one.  A zero or NaN q (a point on a node, a NaN
// point) makes the results infinite or NaN, and so does a subnormal q whose
// reciprocal overflows; the caller's test of its tile sums catches them, as
// it catches the infinite reciprocal of a zero difference with G = 1.  (An
// infinite q cannot occur inside the binary32 domain: differences are at
// most twice the node span, 2^21, so a product of four stays below 2^84.)
// The one unflagged case, a subnormal q in [2^-128, 2^-126) with a finite
// reciprocal, rounds q to 2^-22 relative instead of 2^-24.
__device__ __forceinline__ void group4_reciprocals32(float& d0, float& d1, float& d2, float& d3) {
  const float q01 = d0 * d1, q23 = d2 * d3;
  const float q = q01 * q23;
  const float y = __builtin_amdgcn_rcpf(q);
  const float y01 = y * q23, y23 = y * q01;
  const float t0 = y01 * d1, t1 = y01 * d0, t2 = y23 * d3, t3 = y23 * d2;
  d0 = t0;
  d1 = t1;
  d2 = t2;
  d3 = t3;
}

// Sums of one block over the split node table s4[0, n_pad) (n_pad a multiple
// of 8): the block stages kStage records at a time in LDS (double
// buffered), every wave reads them back with uniform addresses, and each
// lane accumulates its P points in binary32 tile sums promoted to binary64
// every kTile nodes.  G = 1 takes one v_rcp_f32 per difference; G = 4 the
// simultaneous inversion of the four differences of each node quad
// (group4_reciprocals32).  A tile sum that is not finite -- a point on or
// extremely close to a node, a NaN point -- flags the lane for the exact
// path.  B (weights that alternate in sign, see accumulate_f64_blocks): each
// tile is a block, its sums E (first and third record of every quad) and O
// (second and fourth) give D += E + O and A += |E - O| with one multiply-
// add per pair; the tile around the point is corrected afterwards
// (split_tile_fix).  Must be called by all threads of the block.
template <int P, bool R, bool L, int G = 1, bool B = false>
__device__ __forceinline__ void split_block_sums(float4 (&stage)[2][kStage],
                                                 const float4* __restrict__ s4, int64_t n_pad,
                                                 uint32_t mask, const float (&xh)[P],
                                                 const float (&xl)[P], double (&N)[P],
                                                 double (&D)[P], double (&A)[P], bool (&bad)[P]) {
  static_assert(G == 1 || G == 4, "group size 1 or 4");
  const int tid = threadIdx.x;
  // B: Dt and At hold the tile's E and O
  float Nt[P], Dt[P], At[P];
#pragma unroll
  for (int j = 0; j < P; ++j) Nt[j] = Dt[j] = At[j] = 0.0f;
  if (tid < n_pad) stage[0][tid] = s4[tid];
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < n_pad; k0 += kStage) {
    // prefetch the next stage into the other buffer (last read two stages
    // ago, released by the barrier that ended the previous stage)
    const int64_t kn = k0 + kStage + tid;
    if (kn < n_pad) stage[buf ^ 1][tid] = s4[kn];
    const int cnt = (int)(n_pad - k0 < kStage ? n_pad - k0 : kStage);  // multiple of 8
    for (int i0 = 0; i0 < cnt; i0 += kTile) {
      const int iend = i0 + kTile < cnt ? i0 + kTile : cnt;
      for (int i = i0; i < iend; i += 4) {
        // four nodes at a time, all their P x 4 pairs independent
        float4 rc[4];
        float t[4][P];
#pragma unroll
        for (int q = 0; q < 4; ++q) rc[q] = stage[buf][i + q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) t[q][j] = (xh[j] - rc[q].x) + (xl[j] - rc[q].y);
        if constexpr (G == 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < P; ++j) t[q][j] = __builtin_amdgcn_rcpf(t[q][j]);
        } else {
#pragma unroll
          for (int j = 0; j < P; ++j) group4_reciprocals32(t[0][j], t[1][j], t[2][j], t[3][j]);
        }
        if constexpr (B) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < P; ++j) {
              if (q & 1)
                At[j] = __builtin_fmaf(rc[q].z, t[q][j], At[j]);
              else
                Dt[j] = __builtin_fmaf(rc[q].z, t[q][j], Dt[j]);
              if (R) Nt[j] = __builtin_fmaf(rc[q].w, t[q][j], Nt[j]);
            }
          continue;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) {
            Dt[j] = __builtin_fmaf(rc[q].z, t[q][j], Dt[j]);
            if (R) Nt[j] = __builtin_fmaf(rc[q].w, t[q][j], Nt[j]);
          }
        if (L) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float aw = abs_vop2(rc[q].z, mask);
#pragma unroll
            for (int j = 0; j < P; ++j) At[j] = __builtin_fmaf(aw, abs_vop2(t[q][j], mask), At[j]);
          }
        }
      }
      if constexpr (B) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          bad[j] |= not_finite32(Dt[j]) | not_finite32(At[j]);
          const double e = (double)Dt[j], o = (double)At[j];
          D[j] += e + o;
          if (L) A[j] += fabs(e - o);
          Dt[j] = At[j] = 0.0f;
          if (R) {
            bad[j] |= not_finite32(Nt[j]);
            N[j] += (double)Nt[j];
            Nt[j] = 0.0f;
          }
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < P; ++j) {
        bad[j] |= not_finite32(Dt[j]);
        D[j] += (double)Dt[j];
        Dt[j] = 0.0f;
        if (R) {
          bad[j] |= not_finite32(Nt[j]);
          N[j] += (double)Nt[j];
          Nt[j] = 0.0f;
        }
        if (L) {
          bad[j] |= not_finite32(At[j]);
          A[j] += (double)At[j];
          At[j] = 0.0f;
        }
      }
    }
    __syncthreads();
    buf ^= 1;
  }
}

// The Lebesgue sum A of split_block_sums<..., B = true> corrected for the
// tile (kTile records) that holds nodes on both sides of the point xv (found
// by binary search in the binary64 nodes tx[0, n)): its |E - O|, recomputed
// from the split records s4 with the loop's operations, is replaced by
// sum_k |w_k t_k|.  xv finite and not a node; n_pad (a multiple of 4) ends
// the records, so a table's last tile may be partial, as in the loop.
template <int G>
__device__ __forceinline__ double split_tile_fix(double xv, float xh, float xl,
                                                 const double* __restrict__ tx, int64_t n,
                                                 const float4* __restrict__ s4, int64_t n_pad,
                                                 uint32_t mask, double A) {
  const int64_t j = nodes_below(xv, tx, n);
  if (j == 0 || j >= n || j % kTile == 0) return A;
  const int64_t b = j - j % kTile;
  const int len = (int)(n_pad - b < kTile ? n_pad - b : kTile);
  float E = 0.0f, O = 0.0f, exact = 0.0f;
#pragma unroll 1
  for (int i = 0; i < len; i += 4) {
    float4 rc[4];
    float t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      rc[q] = s4[b + i + q];
      t[q] = (xh - rc[q].x) + (xl - rc[q].y);
    }
    if constexpr (G == 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] = __builtin_amdgcn_rcpf(t[q]);
    } else {
      group4_reciprocals32(t[0], t[1], t[2], t[3]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q & 1)
        O = __builtin_fmaf(rc[q].z, t[q], O);
      else
        E = __builtin_fmaf(rc[q].z, t[q], E);
      exact = __builtin_fmaf(abs_vop2(rc[q].z, mask), abs_vop2(t[q], mask), exact);
    }
  }
  return (A - fabs((double)E - (double)O)) + (double)exact;
}

// Streams the records src[0, count) (count a multiple of 4) through the
// block's double-buffered LDS stage, as split_block_sums does: quad(rc) is
// called for every four consecutive records (rc[4], the same for all lanes:
// wave-uniform LDS reads), and flush(begin, end) after every kTile records
// and after the last one, with the record range of that tile.  Must be
// called by all kStage threads of the block.
template <class Quad, class Flush>
__device__ __forceinline__ void staged_tiles(float4 (&stage)[2][kStage],
                                             const float4* __restrict__ src, int64_t count,
                                             Quad&& quad, Flush&& flush) {
  const int tid = threadIdx.x;
  if (tid < count) stage[0][tid] = src[tid];
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < count; k0 += kStage) {
    const int64_t kn = k0 + kStage + tid;
    if (kn < count) stage[buf ^ 1][tid] = src[kn];
    const int cnt = (int)(count - k0 < kStage ? count - k0 : kStage);
    for (int i0 = 0; i0 < cnt; i0 += kTile) {
      const int iend = i0 + kTile < cnt ? i0 + kTile : cnt;
      for (int i = i0; i < iend; i += 4) {
        float4 rc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rc[q] = stage[buf][i + q];
        quad(rc);
      }
      flush(k0 + i0, k0 + iend);
    }
    __syncthreads();
    buf ^= 1;
  }
}

// ------------------------------------------------------- binary32 domain --
// The split node table of one interpolant: {binary32 head of x_k, binary32
// tail x_k - head, w_k 2^-e, w_k f_k 2^-ef} with 2^e and 2^ef the binary
// exponents of max|w_k| and max|w_k f_k| (multiplying by a power of two is
// exact).  The weighted values get their own scale so that the table does
// not depend on the magnitude of f; the kernels restore it as
// r = 2^(ef - e) N / D, exactly.
//
// The binary32 terms are trusted only inside a domain where every term
// that matters is a normal binary32 number: node span in [2^-20, 2^20],
// nonzero |w_k| >= 2^(e - 100) and nonzero finite |w_k f_k| >= 2^(ef - 100)
// (table), and points no further than one span outside the nodes (point,
// tested by the kernels), so that |t| >= 2^-21 / 2.  A table outside the
// domain is written with NaN weights: every point then takes the binary64
// per-pair path.  Terms of tiny weight that still underflow inside the
// domain are below 2^-100 of the largest term of their sum.
constexpr double kSpanMin = 0x1p-20, kSpanMax = 0x1p20;
constexpr int kWeightRange = 100;

struct SplitScale {
  int e;      // max|w| = m 2^e, 1/2 <= m < 1
  int shift;  // ef - e
  bool ok;    // table inside the binary32 domain
};

// Block-wide (all threads, blockDim.x == 256) reduction over one table of
// n real nodes in [0, n_pad); red is a 4 x 256 LDS scratch.
__device__ inline SplitScale split_table_scale(const double* __restrict__ tx,
                                               const double* __restrict__ tw,
                                               const double* __restrict__ twf, int64_t n,
                                               int64_t n_pad, double (*red)[256]) {
  const int tid = threadIdx.x;
  double mxw = 0.0, mxf = 0.0, mnw = __builtin_inf(), mnf = __builtin_inf();
  for (int64_t k = tid; k < n_pad; k += blockDim.x) {
    const double aw = fabs(tw[k]), af = fabs(twf[k]);
    mxw = fmax(mxw, aw);
    if (aw != 0.0) mnw = fmin(mnw, aw);
    if (__builtin_isfinite(af)) {
      mxf = fmax(mxf, af);
      if (af != 0.0) mnf = fmin(mnf, af);
    }
  }
  red[0][tid] = mxw;
  red[1][tid] = mxf;
  red[2][tid] = mnw;
  red[3][tid] = mnf;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
      red[1][tid] = fmax(red[1][tid], red[1][tid + s]);
      red[2][tid] = fmin(red[2][tid], red[2][tid + s]);
      red[3][tid] = fmin(red[3][tid], red[3][tid + s]);
    }
    __syncthreads();
  }
  SplitScale sc;
  int ef = 0;
  frexp(red[0][0], &sc.e);
  frexp(red[1][0], &ef);
  sc.shift = ef - sc.e;
  const double span = tx[n - 1] - tx[0];
  sc.ok = n >= 2 && span >= kSpanMin && span <= kSpanMax &&
          red[2][0] >= ldexp(1.0, sc.e - kWeightRange) &&
          red[3][0] >= ldexp(1.0, ef - kWeightRange);
  __syncthreads();  // red may be reused by the caller
  return sc;
}

// Conditioning of a split table, decided once at packing: Lebesgue function
// above which a table takes binary64 terms for all its points.  It lies
// below the per-point guard kSplitLambdaGuard, so that few points of a
// table that passes are left to that guard.
constexpr double kSplitWideGuard = 0x1p12;
constexpr int kWideSamples = 64;

// Block-wide (all threads, blockDim.x == 256, records tx/tw wave-uniform):
// 1 in every thread if the Lebesgue function of the table of n nodes
// exceeds kSplitWideGuard (or is not a number) at one of the midpoints of
// kWideSamples intervals spread over it, else 0 (always 0 for n < 2).  The
// samples are evaluated in binary64 with groups of four differences per
// reciprocal; wave w sums the records [w q, (w + 1) q) (q = four-aligned
// quarter of the table rounded up to 4) and the four partial sums are added
// in wave order, so the decision depends only on the n real nodes (padding
// records beyond them add exact zeros): the single and the batched split
// kernels decide alike.  red: LDS scratch of the caller, free on entry.
__device__ inline int split_table_wide(const double* __restrict__ tx,
                                       const double* __restrict__ tw, int64_t n,
                                       double (*red)[256]) {
  if (n < 2) return 0;  // n is uniform over the block
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nr = (n + 3) / 4 * 4, q = ((n + 3) / 4 + 3) / 4 * 4;
  const int64_t k0 = wave * q < nr ? wave * q : nr, k1 = (wave + 1) * q < nr ? (wave + 1) * q : nr;
  const int64_t i = ((int64_t)lane * (n - 1)) / kWideSamples;
  double xp[1] = {tx[i] + 0.5 * (tx[i + 1] - tx[i])}, N[1] = {0.0}, D[1] = {0.0}, A[1] = {0.0};
  bool bad[1] = {false};
  accumulate_f64<1, 4, false, true>(xp, tx, tw, tw, k0, k1, N, D, A, bad);
  red[0][threadIdx.x] = D[0];
  red[1][threadIdx.x] = A[0];
  __syncthreads();
  int wide = 0;
  if (wave == 0) {
    double ds = red[0][lane], as = red[1][lane];
    for (int w = 1; w < 4; ++w) {
      ds += red[0][w * 64 + lane];
      as += red[1][w * 64 + lane];
    }
    wide = !(as <= kSplitWideGuard * fabs(ds));
  }
  return __syncthreads_or(wide);
}

__device__ inline float4 split_record(double xk, double w, double wf, const SplitScale& sc) {
  const float hi = (float)xk;
  const float lo = (float)(xk - (double)hi);
  if (!sc.ok) {
    const float nan = __builtin_nanf("");
    return make_float4(hi, lo, nan, nan);
  }
  return make_float4(hi, lo, (float)ldexp(w, -sc.e), (float)ldexp(wf, -(sc.e + sc.shift)));
}

// Position of the zero-weight padding records of a split table: two node
// spans beyond the last node, out of reach of every point in the binary32
// domain.  (Copies of the last node would give a point next to it the
// product (x - x_last)^4 of a padding quad, which leaves the binary32 range
// below |x - x_last| ~ 3e-10 and sends the lane to the per-pair path.)
__device__ __forceinline__ double split_pad_x(double x_first, double x_last) {
  return x_last + 2.0 * (x_last - x_first);
}

// A point whose binary32 terms are trusted (also false for NaN): within one
// node span of [x_first, x_last].
__device__ __forceinline__ bool in_split_domain(double x, double x_first, double x_last) {
  const double span = x_last - x_first;
  return x >= x_first - span && x <= x_last + span;
}

}  // namespace fhk
