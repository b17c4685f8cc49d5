// Fused second-form evaluation in binary64 (gfx950).
//
// For every point x and node k: delta = x - x_k, t = 1/delta,
//   N += (w_k f_k) t,   D += w_k t,   L += |w_k| |t|,
// then r = N / D and Lambda = L / |D| (Floater & Hormann 2007, barycentric
// form; Lambda is the Lebesgue function sum_k |a_k| / |sum_k a_k|).
//
// Mapping.  A block has four waves, in 4/S groups of S waves.  The S waves
// of a group own the same 64*P points (each lane P of them, strided by 64
// so loads and stores coalesce); wave s of the group walks the s-th of S
// equal slices of the node table, and the S partial sums (N, D, L) are
// added through LDS in wave order at the end, so the result does not depend
// on timing.  S > 1 multiplies the number of waves for a given point count
// (small point sets would otherwise leave SIMDs idle); P > 1 gives each wave
// independent chains to hide latency.  Blocks are always 256 threads: with
// one-wave blocks the per-CU workgroup limit, not registers, would cap the
// resident waves.  Node records are wave-uniform: they arrive through
// scalar loads as SGPR operands.
//
// Reciprocals.  A division costs far more than a multiply (the paper's
// premise for preferring scaling to quotients).  On gfx950 v_rcp_f64 is a
// quarter-rate estimate with about 24.4 correct bits.  Nodes are taken in
// groups of G (4 or 8) and their reciprocals come from one reciprocal of the
// group product (simultaneous inversion): with a product tree
// q_ab = d_a d_b, ..., Q = product of all, y ~ 1/Q (estimate plus one
// Newton step), each 1/d_k is y times the product of the other deltas, read
// off the same tree.  Cost per pair ~ 1 sub + 3 mul + 3 fma + (rcp + 3)/G
// issue slots instead of ~10 with a refined reciprocal per pair; each t
// keeps a relative error of a few units in the last place.
//
// Hits and range.  Q is zero exactly when some delta is zero (an exact hit),
// NaN for a NaN point, infinite or subnormal only for extreme coordinates.
// Such a Q makes the refined reciprocal NaN, hence D; a lane whose D is not
// finite after the node loop is flagged and recomputes its point with the
// exact-hit branch (r = f_j bit-for-bit, Lambda = 1) or one IEEE division
// per pair.  The loop itself holds no test and no branch.
//
// Node pairs (the default launch variants).  Two nodes of a 16-node block
// give one rational term in the block's coordinates, so one reciprocal and
// one multiply-add per sum serve two nodes (pair_math.h: the identity, its
// error bound, the pack's test); the one or two blocks next to each point
// are masked out of the loop and summed node by node afterwards, and a
// block too wide for the bound next to the node spacings around it is
// summed node by node in the loop.
#include "fh_internal.h"
#include "pair_math.h"

namespace fhk {

// Workgroups go to the eight XCDs in turn (linear id modulo 8), each XCD
// with its own L2.  xcd_block maps the linear id g of G to the logical block
// so that each XCD takes one contiguous run of logical blocks: the octet
// variants' results, written to the points' original positions, then fill
// their cache lines inside one L2 (their sorted points keep the chunk of
// original positions they came from), instead of reaching HBM as partial
// lines from eight.  A bijection of 0..G-1.
__device__ __forceinline__ int64_t xcd_block(int64_t g, int64_t G) {
  constexpr int64_t kXcds = 8;
  const int64_t q = G / kXcds, r = G % kXcds;
  const int64_t x = g % kXcds, k = g / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// U > 0: the sums are taken by blocks of U nodes (accumulate_f64_blocks)
// when the table's weights alternate in sign, which *alt says (written by
// the packing); D, hence r, is then the same with and without Lambda.
// PAIRS (U = 16): the blocks are summed by node pairs (accumulate_f64_pairs)
// from the pair records pr and the blocks next to each point node by node
// afterwards (pair_fix_point); when some block of the table failed the
// pack's test (summary words pok), the loop checks each block's flag and
// takes the failing ones node by node.  JKL: the pair terms' J and K are
// staged in LDS first (jk_lds, n_loop doubles; the launch passes that much
// dynamic LDS).
template <int P, int G, int S, bool R, bool L, int U, bool PAIRS, bool JKL, bool OCT>
__device__ __forceinline__ void eval_f64_points(const double* __restrict__ x, int64_t m,
                                                const double* __restrict__ tx,
                                                const double* __restrict__ tw,
                                                const double* __restrict__ twf,
                                                const double* __restrict__ pr,
                                                const uint32_t* __restrict__ pok, int64_t n_pad,
                                                const double* __restrict__ f, int64_t n,
                                                const uint32_t* __restrict__ alt,
                                                double* __restrict__ r, double* __restrict__ lam,
                                                double* jk_lds, const OctetArgs& oa,
                                                int64_t blk) {
  static_assert(!PAIRS || U == kPairBlock, "pair records come in blocks of 16");
  static_assert(PAIRS || !JKL, "LDS staging serves the pair variants");
  constexpr int PG = 4 / S;  // point groups per block
  const int lane = threadIdx.x & 63;
  // wave index, made provably wave-uniform so node loads stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slice = wave % S, pg = wave / S;
  const int64_t base = (blk * PG + pg) * 64 * P + lane;
  double xp[P], N[P], D[P], A[P];
  bool bad[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * 64;
    xp[j] = x[idx < m ? idx : m - 1];
    N[j] = 0.0;
    D[j] = 0.0;
    A[j] = 0.0;
    bad[j] = false;
  }
  // node slice of this wave: the records up to the first multiple of 16 at
  // or after n -- the zero-weight padding beyond it adds nothing and is not
  // visited (n_pad, a multiple of 64, holds it) -- cut into S slices of
  // whole 16-record units (every group and block length divides 16, so
  // variants that differ only in G or U slice alike: a block variant whose
  // weights do not alternate keeps its plain twin's bits), the last one
  // shorter
  constexpr int64_t kUnit = 16;
  static_assert(kUnit % G == 0 && (U == 0 || kUnit % U == 0), "groups and blocks divide 16");
  const int64_t n_loop = (n + kUnit - 1) / kUnit * kUnit;
  const int64_t slice_len = ((n_loop + S - 1) / S + kUnit - 1) / kUnit * kUnit;
  const int64_t k_begin = slice * slice_len < n_loop ? slice * slice_len : n_loop;
  const int64_t k_end = k_begin + slice_len < n_loop ? k_begin + slice_len : n_loop;

  bool blocks = false;
  int32_t rlast[P];
#pragma unroll
  for (int j = 0; j < P; ++j) rlast[j] = -1;
  if constexpr (U > 0) {
    blocks = __builtin_amdgcn_readfirstlane(*alt) != 0;
    if constexpr (PAIRS) {
      if constexpr (JKL) {
        // every thread of the block takes part before any wave branches
        if (blocks) pair_stage_jk(pr, n_loop, jk_lds);
        __syncthreads();
      }
      if (blocks) {
        OctetView ov{};
        if constexpr (OCT) {
          // the smallest and largest of the wave's points (NaN ignored)
          double lo = xp[0], hi = xp[0];
#pragma unroll
          for (int j = 1; j < P; ++j) {
            lo = fmin(lo, xp[j]);
            hi = fmax(hi, xp[j]);
          }
          for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
          }
          ov.rec = oa.rec;
          ov.on = __builtin_amdgcn_readfirstlane(*oa.ok) != 0;
          ov.xmin = uniform_f64(lo);
          ov.xmax = uniform_f64(hi);
        }
        if (pair_table_ok(pok, n_loop))
          accumulate_f64_pairs<P, R, L, JKL, false, OCT>(xp, pr, jk_lds, tx, tw, twf, k_begin,
                                                         k_end, N, D, A, bad, rlast, &ov);
        else
          accumulate_f64_pairs<P, R, L, JKL, true, OCT>(xp, pr, jk_lds, tx, tw, twf, k_begin,
                                                        k_end, N, D, A, bad, rlast, &ov);
      }
    } else if (blocks) {
      accumulate_f64_blocks<P, G, U, R, L>(xp, tx, tw, twf, k_begin, k_end, N, D, A, bad);
    }
  }
  if (!blocks) accumulate_f64<P, G, R, L>(xp, tx, tw, twf, k_begin, k_end, N, D, A, bad);

  if constexpr (S > 1) {
    // fixed-order reduction of the S partial sums of each group through LDS
    __shared__ double red[PG][S - 1][3][64 * P];
    __shared__ int redbad[PG][S - 1][64 * P];
    __shared__ int redmask[PG][S - 1][PAIRS ? 64 * P : 1];
    if (slice > 0) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        red[pg][slice - 1][0][j * 64 + lane] = N[j];
        red[pg][slice - 1][1][j * 64 + lane] = D[j];
        red[pg][slice - 1][2][j * 64 + lane] = A[j];
        redbad[pg][slice - 1][j * 64 + lane] = bad[j];
        if constexpr (PAIRS) redmask[pg][slice - 1][j * 64 + lane] = rlast[j];
      }
    }
    __syncthreads();
    if (slice > 0) return;
#pragma unroll
    for (int s = 0; s < S - 1; ++s) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        N[j] += red[pg][s][0][j * 64 + lane];
        D[j] += red[pg][s][1][j * 64 + lane];
        A[j] += red[pg][s][2][j * 64 + lane];
        bad[j] |= redbad[pg][s][j * 64 + lane] != 0;
        if constexpr (PAIRS) {
          // the last masked block over all slices (-1: none)
          const int32_t rl = redmask[pg][s][j * 64 + lane];
          rlast[j] = rl > rlast[j] ? rl : rlast[j];
        }
      }
    }
  }

  if constexpr (PAIRS) {
    if (blocks) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        // every finite point has a masked block; a NaN point is flagged
        if (!bad[j] && rlast[j] >= 0)
          pair_fix_point<G, R, L>(xp[j], rlast[j], tx, tw, twf, N[j], D[j], A[j]);
        bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
      }
    }
  }

#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + j * 64;
    if (idx >= m) continue;
    double rv, lv;
    if (bad[j]) {
      const PointRL e = eval_point_exact<R, L>(xp[j], tx, tw, f, n);
      rv = e.r;
      lv = e.l;
    } else {
      double a = A[j];
      if constexpr (L && U > 0 && !PAIRS)
        if (blocks) a = lebesgue_block_fix<G, U>(xp[j], tx, tw, n, a);
      rv = N[j] / D[j];
      lv = a / fabs(D[j]);
    }
    // octet launches run over the points sorted: each result goes to the
    // point's original position
    const int64_t dst = OCT ? (int64_t)oa.order[idx] : idx;
    if (R) r[dst] = rv;
    if (L) lam[dst] = lv;
  }
}

template <int P, int G, int S, bool R, bool L, int U, bool PAIRS, bool JKL, bool OCT>
__global__ void __launch_bounds__(256)
    k_eval_f64(const double* __restrict__ x, int64_t m, const double* __restrict__ tx,
               const double* __restrict__ tw, const double* __restrict__ twf,
               const double* __restrict__ pr, const uint32_t* __restrict__ pok, int64_t n_pad,
               const double* __restrict__ f, int64_t n, const uint32_t* __restrict__ alt,
               double* __restrict__ r, double* __restrict__ lam, OctetArgs oa) {
  extern __shared__ double jk_lds[];
  const int64_t blk = OCT ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  eval_f64_points<P, G, S, R, L, U, PAIRS, JKL, OCT>(x, m, tx, tw, twf, pr, pok, n_pad, f, n, alt,
                                                     r, lam, jk_lds, oa, blk);
}

// Several tables on the same points: table blockIdx.y, the points of
// blockIdx.x as in k_eval_f64.  One launch instead of one per table saves
// the drain of each launch's last blocks and the gap before the next.
template <int P, int G, int S, bool R, bool L, int U, bool PAIRS, bool JKL, bool OCT>
__global__ void __launch_bounds__(256)
    k_eval_f64_many(const double* __restrict__ x, int64_t m, int64_t n_pad, int64_t n,
                    EvalMany a) {
  extern __shared__ double jk_lds[];
  int i = blockIdx.y;
  int64_t blk = blockIdx.x;
  if constexpr (OCT) {
    const int64_t l = xcd_block((int64_t)blockIdx.y * gridDim.x + blockIdx.x,
                                (int64_t)gridDim.x * gridDim.y);
    i = (int)(l / gridDim.x);
    blk = l % gridDim.x;
  }
  eval_f64_points<P, G, S, R, L, U, PAIRS, JKL, OCT>(x, m, a.x[i], a.w[i], a.wf[i], a.pr[i],
                                                     a.pok[i], n_pad, a.f[i], n, a.alt[i], a.r[i],
                                                     a.lam[i], jk_lds,
                                                     OctetArgs{a.oc[i], a.ook[i], a.order}, blk);
}

// Dynamic LDS of a pair variant's launch: J and K of the node range when it
// is at most kPairLdsRecords records (then the JKL kernel runs), else 0.
static size_t pair_lds_bytes(int64_t n) {
  const int64_t n_loop = round_up(n, kPairBlock);
  return n_loop <= kPairLdsRecords ? sizeof(double) * (size_t)n_loop : 0;
}

template <int P, int G, int S, int U, bool PAIRS, bool JKL, bool OCT>
static hipError_t launch_many_k(const double* x, int64_t m, int64_t n, int64_t n_pad,
                                const EvalMany& a, int32_t K, bool r, bool lam, size_t lds,
                                hipStream_t s) {
  const int64_t per = 64LL * P * (4 / S);  // points per block
  const dim3 grid((unsigned)((m + per - 1) / per), (unsigned)K), block(256);
  if (r && lam)
    k_eval_f64_many<P, G, S, true, true, U, PAIRS, JKL, OCT>
        <<<grid, block, lds, s>>>(x, m, n_pad, n, a);
  else if (r)
    k_eval_f64_many<P, G, S, true, false, U, PAIRS, JKL, OCT>
        <<<grid, block, lds, s>>>(x, m, n_pad, n, a);
  else
    k_eval_f64_many<P, G, S, false, true, U, PAIRS, JKL, OCT>
        <<<grid, block, lds, s>>>(x, m, n_pad, n, a);
  return hipGetLastError();
}

template <int P, int G, int S, int U, bool PAIRS, bool OCT>
static hipError_t launch_many_v(const double* x, int64_t m, int64_t n, int64_t n_pad,
                                const EvalMany& a, int32_t K, bool r, bool lam, hipStream_t s) {
  const size_t lds = PAIRS ? pair_lds_bytes(n) : 0;
  if constexpr (PAIRS)
    if (lds > 0)
      return launch_many_k<P, G, S, U, true, true, OCT>(x, m, n, n_pad, a, K, r, lam, lds, s);
  return launch_many_k<P, G, S, U, PAIRS, false, OCT>(x, m, n, n_pad, a, K, r, lam, 0, s);
}

template <int P, int G, int S, int U, bool PAIRS, bool JKL, bool OCT>
static hipError_t launch_k(const double* x, int64_t m, const NodeTable& t, int64_t n,
                           const uint32_t* alt, double* r, double* lam, size_t lds,
                           const OctetArgs& oa, hipStream_t s) {
  const int64_t per = 64LL * P * (4 / S);  // points per block
  const dim3 grid((unsigned)((m + per - 1) / per)), block(256);
  if (r && lam)
    k_eval_f64<P, G, S, true, true, U, PAIRS, JKL, OCT><<<grid, block, lds, s>>>(
        x, m, t.x, t.w, t.wf, t.pr, t.pok, t.n_pad, t.f, n, alt, r, lam, oa);
  else if (r)
    k_eval_f64<P, G, S, true, false, U, PAIRS, JKL, OCT><<<grid, block, lds, s>>>(
        x, m, t.x, t.w, t.wf, t.pr, t.pok, t.n_pad, t.f, n, alt, r, lam, oa);
  else
    k_eval_f64<P, G, S, false, true, U, PAIRS, JKL, OCT><<<grid, block, lds, s>>>(
        x, m, t.x, t.w, t.wf, t.pr, t.pok, t.n_pad, t.f, n, alt, r, lam, oa);
  return hipGetLastError();
}

template <int P, int G, int S, int U, bool PAIRS, bool OCT>
static hipError_t launch_v(const double* x, int64_t m, const NodeTable& t, int64_t n,
                           const uint32_t* alt, double* r, double* lam, const OctetArgs& oa,
                           hipStream_t s) {
  const size_t lds = PAIRS ? pair_lds_bytes(n) : 0;
  if constexpr (PAIRS)
    if (lds > 0)
      return launch_k<P, G, S, U, true, true, OCT>(x, m, t, n, alt, r, lam, lds, oa, s);
  return launch_k<P, G, S, U, PAIRS, false, OCT>(x, m, t, n, alt, r, lam, 0, oa, s);
}

// Variant table: id -> (points per lane P, group size G, node split S,
// Lebesgue block U; U = 0: plain sums, node pairs: 1 for sums by node pairs
// in blocks of U = 16, G then the group of the node-by-node blocks, 2 for
// node pairs and octets: the launch sorts the points by the block of their
// neighbouring nodes and sums the blocks far from a point by octets).
#define FH_F64_VARIANTS(X)                                                                    \
  X(0, 1, 4, 1, 0, 0) X(1, 2, 4, 1, 0, 0) X(2, 4, 4, 1, 0, 0) X(3, 1, 8, 1, 0, 0)             \
  X(4, 2, 8, 1, 0, 0) X(5, 4, 8, 1, 0, 0) X(6, 1, 4, 4, 0, 0) X(7, 2, 4, 4, 0, 0)             \
  X(8, 4, 4, 4, 0, 0) X(9, 1, 8, 4, 0, 0) X(10, 2, 8, 4, 0, 0) X(11, 4, 8, 4, 0, 0)           \
  X(12, 1, 8, 2, 0, 0) X(13, 2, 8, 2, 0, 0) X(14, 4, 8, 2, 0, 0) X(15, 1, 8, 4, 16, 0)        \
  X(16, 2, 8, 4, 16, 0) X(17, 1, 8, 2, 16, 0) X(18, 2, 8, 2, 16, 0) X(19, 1, 8, 2, 16, 1)     \
  X(20, 2, 8, 2, 16, 1) X(21, 2, 8, 4, 16, 1) X(22, 4, 8, 2, 16, 1) X(23, 2, 8, 1, 16, 1)     \
  X(24, 4, 8, 1, 16, 1) X(25, 4, 8, 2, 16, 2) X(26, 2, 8, 2, 16, 2)

int f64_variant_count() {
#define FH_COUNT(id, p, g, s, u, pairs) +1
  return 0 FH_F64_VARIANTS(FH_COUNT);
#undef FH_COUNT
}

void f64_variant_shape(int id, int* p, int* g, int* s) {
  switch (id) {
#define FH_SHAPE(vid, vp, vg, vs, vu, vpairs) \
  case vid:                                   \
    *p = vp;                                  \
    *g = vg;                                  \
    *s = vs;                                  \
    return;
    FH_F64_VARIANTS(FH_SHAPE)
#undef FH_SHAPE
    default: *p = *g = *s = 0;
  }
}

int f64_variant_block(int id) {
  switch (id) {
#define FH_BLOCK(vid, vp, vg, vs, vu, vpairs) \
  case vid: return vu;
    FH_F64_VARIANTS(FH_BLOCK)
#undef FH_BLOCK
    default: return 0;
  }
}

bool f64_variant_pairs(int id) {
  switch (id) {
#define FH_PAIRS(vid, vp, vg, vs, vu, vpairs) \
  case vid: return vpairs != 0;
    FH_F64_VARIANTS(FH_PAIRS)
#undef FH_PAIRS
    default: return false;
  }
}

bool f64_variant_octets(int id) {
  switch (id) {
#define FH_OCTETS(vid, vp, vg, vs, vu, vpairs) \
  case vid: return vpairs == 2;
    FH_F64_VARIANTS(FH_OCTETS)
#undef FH_OCTETS
    default: return false;
  }
}

int f64_variant_octet_twin(int id) {
  if (!f64_variant_octets(id)) return id;
  int p, g, s;
  f64_variant_shape(id, &p, &g, &s);
  for (int k = 0; k < f64_variant_count(); ++k) {
    int kp, kg, ks;
    f64_variant_shape(k, &kp, &kg, &ks);
    if (f64_variant_pairs(k) && !f64_variant_octets(k) && kp == p && kg == g && ks == s) return k;
  }
  return id;
}

hipError_t launch_eval_f64(const double* x, int64_t m, const NodeTable& t, int64_t n,
                           const uint32_t* alt, double* r, double* lam, const EvalConfig& cfg,
                           const OctetArgs& oa, hipStream_t s) {
  if (m == 0) return hipSuccess;
  switch (cfg.variant) {
#define FH_CASE(vid, vp, vg, vs, vu, vpairs) \
  case vid:                                   \
    return launch_v<vp, vg, vs, vu, vpairs != 0, vpairs == 2>(x, m, t, n, alt, r, lam, oa, s);
    FH_F64_VARIANTS(FH_CASE)
#undef FH_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval_f64_many(const double* x, int64_t m, int64_t n, int64_t n_pad,
                                const EvalMany& a, int32_t K, bool r, bool lam,
                                const EvalConfig& cfg, hipStream_t s) {
  if (m == 0 || K == 0) return hipSuccess;
  switch (cfg.variant) {
#define FH_CASE(vid, vp, vg, vs, vu, vpairs) \
  case vid:                                   \
    return launch_many_v<vp, vg, vs, vu, vpairs != 0, vpairs == 2>(x, m, n, n_pad, a, K, r, lam, s);
    FH_F64_VARIANTS(FH_CASE)
#undef FH_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fhk
