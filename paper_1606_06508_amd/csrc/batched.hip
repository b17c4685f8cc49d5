// Batched evaluation: many interpolants of uneven n and d in one captured
// HIP graph (gfx950).
//
// Layout.  The caller's arrays are CSR: instance i owns nodes/values
// [noff_i, noff_i + n_i) and points/outputs [poff_i, poff_i + m_i).  The
// batch builds one concatenated node table (x, w, w f, f in binary64 and the
// binary32 split records), each instance padded to a multiple of 8 records
// with zero-weight copies of its last node.
//
// Work.  A work item is one strip of consecutive points of one instance:
// Q passes of the block, each pass 64 * P * (4 / S) points (P points per
// lane, S waves splitting the node range of each group of 64 * P points).
// Items are ordered longest first (by the instance's padded node count,
// i.e. the cost of a strip), and a persistent grid sized to the resident
// capacity of the device pulls them from an atomic counter: big strips
// start first, small ones fill the tail.  Inside a pass the block runs the
// node loops of the single-interpolant kernels (binary64: each wave streams
// its slice of the instance's node records through scalar loads; split: the
// block stages them in LDS).
//
// Launch variants (the autotuner's choice per batch shape): points per lane
// P, node split S, the binary64 Lebesgue block U (0 = plain sums; 16 = sums
// by node blocks, one multiply-add per pair for D and the Lebesgue sum, the
// block around each point corrected afterwards; the batch's weights are the
// library's, which alternate in sign), passes per strip Q, and for U = 16
// sums by node pairs (pair_math.h; an instance with a block that fails the
// pair test takes the node-block sums).  Binary64 variants with U = 16 pad
// each instance to a multiple of 16 records, the others to 8.  The split kernel always takes its sums by node tiles (with
// or without Lambda, so r does not depend on it); its variants are P and Q.
//
// Graph.  fh_batch_create captures, on a private stream: a one-thread kernel
// that resets the item counter (a kernel rather than a memset node), the
// weight/packing pass for all instances, the split or node-pair packing pass
// if needed, and the persistent evaluation kernel.  fh_eval_batched is one
// hipGraphLaunch.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "fh_internal.h"
#include "pair_math.h"
#include "split_math.h"
#include "weight_math.h"

namespace fhk {

struct InstDesc {
  int64_t noff, n, toff, n_pad, poff, m;
  int32_t d, strips;
  int32_t shift;       // split: ef - e of the instance's table (written by its packing)
  int32_t wide;        // split: 1 if the instance takes binary64 terms (written by its packing)
  int32_t pairs_bad;   // binary64 pair variants: blocks of the instance that failed the
                       // pair test (written by k_batch_pack_pairs; 0: the pair loop
                       // takes no per-block test)
  int32_t reserved;
};

constexpr int64_t kBatchPad = 8;

// ------------------------------------------------------------- packing --
__global__ void __launch_bounds__(256)
    k_batch_pack(const InstDesc* __restrict__ inst, const int64_t* __restrict__ toff, int32_t count,
                 int64_t total, const double* __restrict__ nodes, const double* __restrict__ values,
                 double* __restrict__ tx, double* __restrict__ tw, double* __restrict__ twf,
                 double* __restrict__ tf, uint32_t* status) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  // instance of table entry e: toff[i] <= e < toff[i + 1]
  int32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  const InstDesc ds = inst[lo];
  const int64_t k = e - ds.toff;
  const double* x = nodes + ds.noff;
  if (k >= ds.n) {
    tx[e] = x[ds.n - 1];
    tw[e] = 0.0;
    twf[e] = 0.0;
    tf[e] = 0.0;
    return;
  }
  uint32_t flags = node_checks(x, ds.n, k);
  const double wk = node_weight(x, ds.n, ds.d, k, &flags);
  const double fk = values[ds.noff + k];
  tx[e] = x[k];
  tw[e] = wk;
  twf[e] = wk * fk;
  tf[e] = fk;
  if (flags) atomicOr(status, flags);
}

// one block per instance: exponent of max|w| of that instance, then its
// binary32 records (see k_pack_split for the scaling argument), then its
// conditioning (split_table_wide): an instance too ill-conditioned for
// binary32 terms, or outside the binary32 domain, is marked wide and every
// point of it is evaluated with binary64 terms (the per-point guard would
// send most of them there one lane at a time).
__global__ void __launch_bounds__(256)
    k_batch_pack_split(InstDesc* __restrict__ inst, const double* __restrict__ tx,
                       const double* __restrict__ tw, const double* __restrict__ twf,
                       float4* __restrict__ s4) {
  __shared__ double red[4][256];
  const InstDesc ds = inst[blockIdx.x];
  const SplitScale sc =
      split_table_scale(tx + ds.toff, tw + ds.toff, twf + ds.toff, ds.n, ds.n_pad, red);
  if (threadIdx.x == 0) inst[blockIdx.x].shift = sc.shift;
  const double pad = split_pad_x(tx[ds.toff], tx[ds.toff + ds.n - 1]);
  for (int64_t k = threadIdx.x; k < ds.n_pad; k += blockDim.x) {
    const int64_t e = ds.toff + k;
    s4[e] = split_record(k < ds.n ? tx[e] : pad, tw[e], twf[e], sc);
  }
  const int wide = split_table_wide(tx + ds.toff, tw + ds.toff, ds.n, red) | !sc.ok;
  if (threadIdx.x == 0) inst[blockIdx.x].wide = wide;
}

// One block per instance: the node-pair records of its blocks of 16 records
// (pair_record_header / pair_record_pair, one thread per block of records)
// and the number of blocks that failed the pair test.
__global__ void __launch_bounds__(256)
    k_batch_pack_pairs(InstDesc* __restrict__ inst, const double* __restrict__ tx,
                       const double* __restrict__ tw, const double* __restrict__ twf,
                       double* __restrict__ tpr) {
  __shared__ int bad_blocks;
  if (threadIdx.x == 0) bad_blocks = 0;
  __syncthreads();
  const InstDesc ds = inst[blockIdx.x];
  const double* x = tx + ds.toff;
  int mine = 0;
  for (int64_t b = threadIdx.x; b * kPairBlock < ds.n_pad; b += blockDim.x) {
    const int64_t k0 = b * kPairBlock;
    double* rec = tpr + (ds.toff / kPairBlock + b) * kPairRec;
    for (int t = 0; t < 8; ++t) pair_record_pair(x, ds.n, k0, tw + ds.toff + k0, twf + ds.toff + k0, t, rec);
    mine += pair_record_header(x, ds.n, k0, tw + ds.toff + k0, twf + ds.toff + k0, rec) ? 0 : 1;
  }
  if (mine) atomicAdd(&bad_blocks, mine);
  __syncthreads();
  if (threadIdx.x == 0) inst[blockIdx.x].pairs_bad = bad_blocks;
}

__global__ void k_batch_reset(uint32_t* counter) { *counter = 0u; }

// ------------------------------------------------------ persistent eval --
// Pull the next item; all threads of the block get the same (uniform) id.
__device__ __forceinline__ int next_item(uint32_t* counter, int* s_item) {
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(*s_item);
  __syncthreads();
  return item;
}

// Binary64: wave (slice, pg) of the block owns the 64 * P points pg of the
// pass and the node slice `slice` (whole node groups, or whole blocks of U
// records); the S partial sums meet in LDS in wave order.  PAIRS (U = 16):
// every instance is summed by node pairs from its records in tpr (J and K
// copied to VGPRs), the blocks next to each point node by node afterwards,
// as in k_eval_f64; in an instance with blocks that failed the pair test
// (pairs_bad) the loop takes those blocks node by node.
template <int P, int G, int S, bool R, bool L, int U, bool PAIRS>
__global__ void __launch_bounds__(256)
    k_batch_f64(const InstDesc* __restrict__ inst, const int2* __restrict__ items, int n_items,
                int32_t passes, uint32_t* counter, const double* __restrict__ x,
                double* __restrict__ r, double* __restrict__ lam, const double* __restrict__ tx,
                const double* __restrict__ tw, const double* __restrict__ twf,
                const double* __restrict__ tf, const double* __restrict__ tpr) {
  static_assert(!PAIRS || U == kPairBlock, "pair records come in blocks of 16");
  constexpr int PG = 4 / S;  // point groups per block
  constexpr int64_t kPass = 64LL * P * PG;
  constexpr int64_t kUnit = U > 0 ? U : G;
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slice = wave % S, pg = wave / S;
  for (;;) {
    const int item = next_item(counter, &s_item);
    if (item >= n_items) break;
    const int2 it = items[item];
    const InstDesc ds = inst[__builtin_amdgcn_readfirstlane(it.x)];
    const int64_t strip = __builtin_amdgcn_readfirstlane(it.y);
    const double* px = x + ds.poff;
    const double *ix = tx + ds.toff, *iw = tw + ds.toff, *iwf = twf + ds.toff, *iff = tf + ds.toff;
    const bool mixed = PAIRS && __builtin_amdgcn_readfirstlane(ds.pairs_bad) != 0;
    const double* ipr = PAIRS ? tpr + (ds.toff / kPairBlock) * kPairRec : tpr;
    // node slice of this wave: whole units, the last slices possibly shorter
    const int64_t units = ds.n_pad / kUnit;
    const int64_t per_slice = (units + S - 1) / S;
    const int64_t u0 = slice * per_slice < units ? slice * per_slice : units;
    const int64_t u1 = (slice + 1) * per_slice < units ? (slice + 1) * per_slice : units;
    const int64_t first = strip * passes * kPass;
    for (int q = 0; q < passes; ++q) {
      const int64_t pass0 = first + q * kPass;
      if (pass0 >= ds.m) break;  // uniform over the block
      const int64_t base = pass0 + pg * 64 * P + lane;
      double xp[P], N[P], D[P], A[P];
      bool bad[P];
      int32_t rlast[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int64_t idx = base + j * 64;
        xp[j] = px[idx < ds.m ? idx : ds.m - 1];
        N[j] = D[j] = A[j] = 0.0;
        bad[j] = false;
        rlast[j] = -1;
      }
      if constexpr (PAIRS) {
        if (mixed)
          accumulate_f64_pairs<P, R, L, false, true>(xp, ipr, ipr, ix, iw, iwf, u0 * kUnit,
                                                     u1 * kUnit, N, D, A, bad, rlast);
        else
          accumulate_f64_pairs<P, R, L, false, false>(xp, ipr, ipr, ix, iw, iwf, u0 * kUnit,
                                                      u1 * kUnit, N, D, A, bad, rlast);
      } else if constexpr (U > 0)
        accumulate_f64_blocks<P, G, U, R, L>(xp, ix, iw, iwf, u0 * kUnit, u1 * kUnit, N, D, A,
                                             bad);
      else
        accumulate_f64<P, G, R, L>(xp, ix, iw, iwf, u0 * kUnit, u1 * kUnit, N, D, A, bad);
      if constexpr (S > 1) {
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
        if (slice == 0) {
#pragma unroll
          for (int h = 0; h < S - 1; ++h) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
              N[j] += red[pg][h][0][j * 64 + lane];
              D[j] += red[pg][h][1][j * 64 + lane];
              A[j] += red[pg][h][2][j * 64 + lane];
              bad[j] |= redbad[pg][h][j * 64 + lane] != 0;
              if constexpr (PAIRS) {
                const int32_t rl = redmask[pg][h][j * 64 + lane];
                rlast[j] = rl > rlast[j] ? rl : rlast[j];
              }
            }
          }
        }
        __syncthreads();  // the partial sums are read: the next pass may write
        if (slice > 0) continue;
      }
      if constexpr (PAIRS) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!bad[j] && rlast[j] >= 0)
            pair_fix_point<G, R, L>(xp[j], rlast[j], ix, iw, iwf, N[j], D[j], A[j]);
          bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
        }
      }
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int64_t idx = base + j * 64;
        if (idx >= ds.m) continue;
        double rv, lv;
        if (bad[j]) {
          const PointRL e = eval_point_exact<R, L>(xp[j], ix, iw, iff, ds.n);
          rv = e.r;
          lv = e.l;
        } else {
          double a = A[j];
          if constexpr (L && U > 0 && !PAIRS) a = lebesgue_block_fix<G, U>(xp[j], ix, iw, ds.n, a);
          rv = N[j] / D[j];
          lv = a / fabs(D[j]);
        }
        if (R) r[ds.poff + idx] = rv;
        if (L) lam[ds.poff + idx] = lv;
      }
    }
  }
}

template <int P, bool R, bool L>
__global__ void __launch_bounds__(kStage)
    k_batch_split(const InstDesc* __restrict__ inst, const int2* __restrict__ items, int n_items,
                  int32_t passes, uint32_t* counter, const double* __restrict__ x,
                  double* __restrict__ r, double* __restrict__ lam, const float4* __restrict__ s4,
                  const double* __restrict__ tx, const double* __restrict__ tw,
                  const double* __restrict__ twf, const double* __restrict__ tf) {
  constexpr int64_t kPass = (int64_t)kStage * P;
  __shared__ float4 stage[2][kStage];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const uint32_t mask =
      0x7fffffffu ^ (__builtin_amdgcn_mbcnt_lo(~0u, 0u) & (uint32_t)(n_items >> 30));
  for (;;) {
    const int item = next_item(counter, &s_item);
    if (item >= n_items) break;
    const int2 it = items[item];
    const InstDesc ds = inst[__builtin_amdgcn_readfirstlane(it.x)];
    const int64_t strip = __builtin_amdgcn_readfirstlane(it.y);
    const double* px = x + ds.poff;
    const double x_first = tx[ds.toff], x_last = tx[ds.toff + ds.n - 1];
    const int64_t first = strip * passes * kPass;
    for (int q = 0; q < passes; ++q) {
      const int64_t pass0 = first + q * kPass;
      if (pass0 >= ds.m) break;  // uniform over the block
      const int64_t base = pass0 + tid;
      double xp[P], N[P], D[P], A[P];
      float xh[P], xl[P];
      bool bad[P], wide64[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int64_t idx = base + j * kStage;
        xp[j] = px[idx < ds.m ? idx : ds.m - 1];
        xh[j] = (float)xp[j];
        xl[j] = (float)(xp[j] - (double)xh[j]);
        N[j] = D[j] = A[j] = 0.0;
        wide64[j] = !in_split_domain(xp[j], x_first, x_last);
        bad[j] = wide64[j];
      }
      const double *ix = tx + ds.toff, *iw = tw + ds.toff, *iwf = twf + ds.toff;
      if (ds.wide) {
        // an instance too ill-conditioned for binary32 terms: binary64 terms
        // for all its points (the per-point operations of eval_point_f64)
#pragma unroll
        for (int j = 0; j < P; ++j) bad[j] = wide64[j] = false;
        accumulate_f64<P, 4, R, L>(xp, ix, iw, iwf, 0, ds.n_pad, N, D, A, bad);
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int64_t idx = base + j * kStage;
          if (idx >= ds.m || bad[j]) continue;
          if (R) r[ds.poff + idx] = N[j] / D[j];
          if (L) lam[ds.poff + idx] = A[j] / fabs(D[j]);
        }
      } else {
        // the Lebesgue sum is always accumulated: the conditioning guard
        // needs it
        split_block_sums<P, R, true, 4, true>(stage, s4 + ds.toff, ds.n_pad, mask, xh, xl, N, D,
                                              A, bad);
        // as in k_eval_split: points that pass the guard, then points for
        // binary64 terms, then the exact branch for sums that are not finite
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int64_t idx = base + j * kStage;
          if (idx >= ds.m || bad[j]) continue;
          const double a = split_tile_fix<4>(xp[j], xh[j], xl[j], ix, ds.n, s4 + ds.toff,
                                             ds.n_pad, mask, A[j]);
          if (!(a <= kSplitLambdaGuard * fabs(D[j]))) {
            bad[j] = wide64[j] = true;
            continue;
          }
          if (R) r[ds.poff + idx] = ldexp(N[j] / D[j], ds.shift);
          if (L) lam[ds.poff + idx] = a / fabs(D[j]);
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int64_t idx = base + j * kStage;
          if (idx >= ds.m || !wide64[j]) continue;
          const PointRLF e = eval_point_f64<R, L>(xp[j], ix, iw, iwf, ds.n_pad);
          if (e.flagged) continue;
          bad[j] = false;
          if (R) r[ds.poff + idx] = e.r;
          if (L) lam[ds.poff + idx] = e.l;
        }
      }
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int64_t idx = base + j * kStage;
        if (idx >= ds.m || !bad[j]) continue;
        const PointRL ex = eval_point_exact<R, L>(xp[j], ix, iw, tf + ds.toff, ds.n);
        if (R) r[ds.poff + idx] = ex.r;
        if (L) lam[ds.poff + idx] = ex.l;
      }
      __syncthreads();  // the next pass's staging reuses the LDS buffers
    }
  }
}

// Variant tables.  Binary64: id -> (points per lane P, group G, node split
// S, Lebesgue block U, passes per strip Q, node pairs).  Split: id -> (P, Q),
// with node quads inverted together (G = 4) and sums by 32-node tiles.
#define FH_BATCH_F64_VARIANTS(X)                                                               \
  X(0, 1, 8, 1, 0, 1, 0) X(1, 2, 8, 1, 0, 1, 0) X(2, 4, 8, 1, 0, 1, 0)                        \
  X(3, 1, 8, 2, 0, 1, 0) X(4, 2, 8, 2, 0, 1, 0) X(5, 4, 8, 2, 0, 1, 0)                        \
  X(6, 1, 8, 1, 16, 1, 0) X(7, 2, 8, 1, 16, 1, 0) X(8, 4, 8, 1, 16, 1, 0)                     \
  X(9, 1, 8, 2, 16, 1, 0) X(10, 2, 8, 2, 16, 1, 0) X(11, 4, 8, 2, 16, 1, 0)                   \
  X(12, 1, 8, 1, 0, 4, 0) X(13, 2, 8, 1, 0, 4, 0) X(14, 4, 8, 1, 0, 4, 0)                     \
  X(15, 2, 8, 2, 0, 4, 0) X(16, 2, 8, 1, 16, 4, 0) X(17, 4, 8, 1, 16, 4, 0)                   \
  X(18, 2, 8, 1, 16, 1, 1) X(19, 4, 8, 1, 16, 1, 1) X(20, 2, 8, 2, 16, 1, 1)                  \
  X(21, 4, 8, 2, 16, 1, 1) X(22, 2, 8, 1, 16, 4, 1) X(23, 4, 8, 1, 16, 4, 1)
#define FH_BATCH_SPLIT_VARIANTS(X) \
  X(0, 1, 1) X(1, 2, 1) X(2, 4, 1) X(3, 8, 1) X(4, 1, 4) X(5, 2, 4) X(6, 4, 4) X(7, 8, 4)

struct BatchShape {
  int p, g, s, u, q;
  bool pairs;
};

BatchShape batch_shape(int id, bool split) {
  if (split) {
    switch (id) {
#define FH_SHAPE(vid, vp, vq) \
  case vid: return {vp, 4, 1, kTile, vq, false};
      FH_BATCH_SPLIT_VARIANTS(FH_SHAPE)
#undef FH_SHAPE
      default: return {0, 0, 0, 0, 0, false};
    }
  }
  switch (id) {
#define FH_SHAPE(vid, vp, vg, vs, vu, vq, vpairs) \
  case vid: return {vp, vg, vs, vu, vq, vpairs != 0};
    FH_BATCH_F64_VARIANTS(FH_SHAPE)
#undef FH_SHAPE
    default: return {0, 0, 0, 0, 0, false};
  }
}

bool batched_variant_pairs(int id, bool split) { return batch_shape(id, split).pairs; }

int batched_variant_count(bool split) {
#define FH_COUNT(...) +1
  return split ? 0 FH_BATCH_SPLIT_VARIANTS(FH_COUNT) : 0 FH_BATCH_F64_VARIANTS(FH_COUNT);
#undef FH_COUNT
}

void batched_variant_shape(int id, int* p, int* g, int* s, bool split) {
  const BatchShape b = batch_shape(id, split);
  *p = b.p;
  *g = b.g;
  *s = b.s;
}

int batched_variant_block(int id, bool split) { return batch_shape(id, split).u; }

int64_t batched_variant_strip(int id, bool split) {
  const BatchShape b = batch_shape(id, split);
  return split ? (int64_t)kStage * b.p * b.q : 64LL * b.p * (4 / (b.s > 0 ? b.s : 1)) * b.q;
}

}  // namespace fhk

using namespace fhk;

struct fh_batch {
  int32_t count = 0, prec = 0, variant = 0, passes = 1;
  int device = 0;
  int64_t total_pad = 0, n_items = 0, strip_pts = 0;
  void* mem = nullptr;
  InstDesc* inst = nullptr;
  int64_t* toff = nullptr;
  int2* items = nullptr;
  uint32_t* ctrl = nullptr;  // [0] item counter, [1] sticky status bits
  double *tx = nullptr, *tw = nullptr, *twf = nullptr, *tf = nullptr;
  double* tpr = nullptr;  // node-pair records (binary64 pair variants)
  float4* s4 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

using F64Kernel = void (*)(const InstDesc*, const int2*, int, int32_t, uint32_t*, const double*,
                           double*, double*, const double*, const double*, const double*,
                           const double*, const double*);
using SplitKernel = void (*)(const InstDesc*, const int2*, int, int32_t, uint32_t*,
                             const double*, double*, double*, const float4*, const double*,
                             const double*, const double*, const double*);

template <int P, int G, int S, int U, bool PAIRS>
F64Kernel f64_kernel(bool r, bool l) {
  return r && l ? k_batch_f64<P, G, S, true, true, U, PAIRS>
                : (r ? k_batch_f64<P, G, S, true, false, U, PAIRS>
                     : k_batch_f64<P, G, S, false, true, U, PAIRS>);
}

F64Kernel pick_f64(int id, bool r, bool l) {
  switch (id) {
#define FH_CASE(vid, vp, vg, vs, vu, vq, vpairs) \
  case vid: return f64_kernel<vp, vg, vs, vu, vpairs != 0>(r, l);
    FH_BATCH_F64_VARIANTS(FH_CASE)
#undef FH_CASE
    default: return nullptr;
  }
}

template <int P>
SplitKernel split_kernel(bool r, bool l) {
  return r && l ? k_batch_split<P, true, true>
                : (r ? k_batch_split<P, true, false> : k_batch_split<P, false, true>);
}

SplitKernel pick_split(int id, bool r, bool l) {
  switch (id) {
#define FH_CASE(vid, vp, vq) \
  case vid: return split_kernel<vp>(r, l);
    FH_BATCH_SPLIT_VARIANTS(FH_CASE)
#undef FH_CASE
    default: return nullptr;
  }
}

// Resident blocks of the batch's kernel on the whole device (-1 on error).
int resident_grid(fh_batch* b, const void* kernel, int block) {
  int per_cu = 0;
  hipDeviceProp_t prop;
  if (kernel == nullptr ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      hipGetDeviceProperties(&prop, b->device) != hipSuccess)
    return -1;
  if (per_cu < 1) per_cu = 1;
  return per_cu * prop.multiProcessorCount;
}

void free_batch(fh_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
}

}  // namespace

extern "C" {

fh_status fh_batch_create(fh_batch** out, int32_t count, const int64_t* n_host,
                          const int32_t* d_host, const int64_t* m_host, const double* nodes_cat,
                          const double* values_cat, const double* x_cat, double* r_cat,
                          double* lambda_cat, int32_t prec, void* stream) {
  if (out == nullptr) return FH_E_ARG;
  *out = nullptr;
  if (count < 1 || !n_host || !d_host || !m_host || !nodes_cat || !values_cat) return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  if (r_cat == nullptr && lambda_cat == nullptr) return FH_E_ARG;
  // host validation and descriptors
  std::vector<InstDesc> inst(count);
  std::vector<int64_t> toff(count + 1, 0);
  int64_t noff = 0, poff = 0, total_pad = 0, total_m = 0, items = 0;
  const int32_t tune_family = prec == FH_FP32_SPLIT ? FH_TUNE_BATCHED_SPLIT : FH_TUNE_BATCHED_FP64;
  for (int32_t i = 0; i < count; ++i) {
    const int64_t n = n_host[i], m = m_host[i];
    const int32_t d = d_host[i];
    if (n < 1 || n > FH_MAX_NODES || m < 0) return FH_E_ARG;
    if (d < 0 || (int64_t)d > n - 1) return FH_E_DEGREE;
    total_m += m;
  }
  if (total_m > 0 && (x_cat == nullptr)) return FH_E_ARG;
  fh_batch* b = new (std::nothrow) fh_batch;
  if (!b) return FH_E_HIP;
  b->count = count;
  b->prec = prec;
  {
    int64_t avg_n = 0;
    for (int32_t i = 0; i < count; ++i) avg_n += n_host[i];
    avg_n = (avg_n + count - 1) / count;
    b->variant = choose_eval_config(tune_family, avg_n, 0, total_m > 0 ? total_m : 1,
                                    r_cat != nullptr, lambda_cat != nullptr)
                     .variant;
  }
  const bool split = prec == FH_FP32_SPLIT;
  const BatchShape shape = batch_shape(b->variant, split);
  b->passes = shape.q;
  b->strip_pts = batched_variant_strip(b->variant, split);
  const int64_t strip_pts = b->strip_pts;
  // binary64 blocks of U records need whole blocks per instance
  const int64_t pad = !split && shape.u > 0 ? shape.u : kBatchPad;
  for (int32_t i = 0; i < count; ++i) {
    InstDesc& ds = inst[i];
    ds.noff = noff;
    ds.n = n_host[i];
    ds.d = d_host[i];
    ds.n_pad = round_up(ds.n, pad);
    ds.toff = total_pad;
    ds.poff = poff;
    ds.m = m_host[i];
    ds.strips = (int32_t)((ds.m + strip_pts - 1) / strip_pts);
    ds.shift = 0;
    ds.wide = 0;
    ds.pairs_bad = 1;  // until k_batch_pack_pairs has looked
    ds.reserved = 0;
    toff[i] = total_pad;
    noff += ds.n;
    poff += ds.m;
    total_pad += ds.n_pad;
    items += ds.strips;
  }
  toff[count] = total_pad;
  if (items > 0x7fffffff) {
    delete b;
    return FH_E_ARG;
  }
  // longest-first work list: instances by decreasing padded node count
  std::vector<int32_t> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t c) { return inst[a].n_pad > inst[c].n_pad; });
  std::vector<int2> work;
  work.reserve(items);
  for (int32_t i : order)
    for (int32_t s = 0; s < inst[i].strips; ++s) work.push_back(make_int2(i, s));
  b->total_pad = total_pad;
  b->n_items = items;

  // one device allocation for everything the batch owns
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t o_inst = take(sizeof(InstDesc) * count);
  const size_t o_toff = take(sizeof(int64_t) * (count + 1));
  const size_t o_items = take(sizeof(int2) * (items > 0 ? items : 1));
  const size_t o_ctrl = take(256);
  const size_t o_tx = take(sizeof(double) * total_pad);
  const size_t o_tw = take(sizeof(double) * total_pad);
  const size_t o_twf = take(sizeof(double) * total_pad);
  const size_t o_tf = take(sizeof(double) * total_pad);
  const size_t o_s4 = prec == FH_FP32_SPLIT ? take(sizeof(float4) * total_pad) : 0;
  const size_t o_pr =
      shape.pairs ? take(sizeof(double) * kPairRec * (size_t)(total_pad / kPairBlock)) : 0;
  if (hipGetDevice(&b->device) != hipSuccess || hipMalloc(&b->mem, off) != hipSuccess) {
    b->mem = nullptr;
    free_batch(b);
    return FH_E_HIP;
  }
  char* base = static_cast<char*>(b->mem);
  b->inst = reinterpret_cast<InstDesc*>(base + o_inst);
  b->toff = reinterpret_cast<int64_t*>(base + o_toff);
  b->items = reinterpret_cast<int2*>(base + o_items);
  b->ctrl = reinterpret_cast<uint32_t*>(base + o_ctrl);
  b->tx = reinterpret_cast<double*>(base + o_tx);
  b->tw = reinterpret_cast<double*>(base + o_tw);
  b->twf = reinterpret_cast<double*>(base + o_twf);
  b->tf = reinterpret_cast<double*>(base + o_tf);
  b->s4 = prec == FH_FP32_SPLIT ? reinterpret_cast<float4*>(base + o_s4) : nullptr;
  b->tpr = shape.pairs ? reinterpret_cast<double*>(base + o_pr) : nullptr;

  hipStream_t user = static_cast<hipStream_t>(stream);
  hipStream_t cs = nullptr;
  hipError_t e = hipSuccess;
  const uint32_t zero_ctrl[2] = {0u, 0u};
  if ((e = hipMemcpyAsync(b->inst, inst.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice,
                          user)) != hipSuccess ||
      (e = hipMemcpyAsync(b->toff, toff.data(), sizeof(int64_t) * (count + 1),
                          hipMemcpyHostToDevice, user)) != hipSuccess ||
      (items > 0 && (e = hipMemcpyAsync(b->items, work.data(), sizeof(int2) * items,
                                        hipMemcpyHostToDevice, user)) != hipSuccess) ||
      (e = hipMemcpyAsync(b->ctrl, zero_ctrl, sizeof(zero_ctrl), hipMemcpyHostToDevice, user)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(user)) != hipSuccess) {
    free_batch(b);
    return FH_E_HIP;
  }

  // capture the whole evaluation into a graph on a private stream
  const bool want_r = r_cat != nullptr, want_l = lambda_cat != nullptr;
  const F64Kernel kf = split ? nullptr : pick_f64(b->variant, want_r, want_l);
  const SplitKernel ks = split ? pick_split(b->variant, want_r, want_l) : nullptr;
  const int block = split ? kStage : 256;
  const int grid =
      resident_grid(b, split ? reinterpret_cast<const void*>(ks) : reinterpret_cast<const void*>(kf),
                    block);
  if (log_enabled())
    std::fprintf(stderr,
                 "[fh] batch of %d instances (%s): variant %d, P %d, S %d, U %d, Q %d, strip %lld "
                 "points, %lld items, grid %d\n",
                 count, split ? "split" : "fp64", b->variant, shape.p, shape.s, shape.u, shape.q,
                 (long long)b->strip_pts, (long long)b->n_items, grid);
  if (grid < 1 || hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    free_batch(b);
    return FH_E_HIP;
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    k_batch_reset<<<1, 1, 0, cs>>>(b->ctrl);
    k_batch_pack<<<(unsigned)((total_pad + 255) / 256), 256, 0, cs>>>(
        b->inst, b->toff, count, total_pad, nodes_cat, values_cat, b->tx, b->tw, b->twf, b->tf,
        b->ctrl + 1);
    if (prec == FH_FP32_SPLIT)
      k_batch_pack_split<<<(unsigned)count, 256, 0, cs>>>(b->inst, b->tx, b->tw, b->twf, b->s4);
    if (shape.pairs)
      k_batch_pack_pairs<<<(unsigned)count, 256, 0, cs>>>(b->inst, b->tx, b->tw, b->twf, b->tpr);
    if (items > 0) {
      const int n_it = (int)b->n_items;
      if (split)
        ks<<<grid, block, 0, cs>>>(b->inst, b->items, n_it, b->passes, b->ctrl, x_cat, r_cat,
                                   lambda_cat, b->s4, b->tx, b->tw, b->twf, b->tf);
      else
        kf<<<grid, block, 0, cs>>>(b->inst, b->items, n_it, b->passes, b->ctrl, x_cat, r_cat,
                                   lambda_cat, b->tx, b->tw, b->twf, b->tf, b->tpr);
      e = hipGetLastError();
    }
    hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    free_batch(b);
    return FH_E_HIP;
  }
  *out = b;
  return FH_OK;
}

fh_status fh_eval_batched(fh_batch* b, void* stream) {
  if (b == nullptr || b->exec == nullptr) return FH_E_ARG;
  return hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? FH_OK
                                                                                  : FH_E_HIP;
}

int32_t fh_batch_variant(const fh_batch* b) { return b ? b->variant : -1; }

int64_t fh_batch_strip_points(const fh_batch* b) { return b ? b->strip_pts : -1; }

fh_status fh_batch_destroy(fh_batch* b) {
  free_batch(b);
  return FH_OK;
}

fh_status fh_batch_status(fh_batch* b, void* stream, uint32_t* bits_out) {
  if (b == nullptr || bits_out == nullptr) return FH_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return FH_E_HIP;
  uint32_t bits = 0;
  if (hipMemcpy(&bits, b->ctrl + 1, sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess)
    return FH_E_HIP;
  if (bits) {
    const uint32_t zero = 0;
    if (hipMemcpy(b->ctrl + 1, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
      return FH_E_HIP;
  }
  *bits_out = bits;
  if (bits & FH_FLAG_NONFINITE) return FH_E_NONFINITE;
  if (bits & FH_FLAG_NODES) return FH_E_NODES;
  if (bits & FH_FLAG_RANGE) return FH_E_RANGE;
  return FH_OK;
}

}  // extern "C"
