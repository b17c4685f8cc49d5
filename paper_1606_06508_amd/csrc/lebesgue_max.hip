// Lebesgue constant of an FH interpolant on gfx950: the largest value of
// the Lebesgue function Lambda(x) = sum_k |a_k| / |sum_k a_k| on every
// interval [x_k, x_{k+1}] (Lambda = 1 at the nodes, so the constant is the
// largest of these), searched for by sampling and zooming in.
//
// The search, per interval (a plain grid zoom):
//   a round samples S interior points of the bracket [lo, hi],
//     h = (hi - lo) / (S + 1),  t_i = lo + (i + 1) h   (i = 0..S-1),
//   with the product and the sum rounded separately (no contraction), so the
//   sample points are the same bits on every IEEE machine;
//   i* = the first index of the largest sampled Lambda (NaN never counts;
//   if no sample is a number the bracket stays and nothing is recorded);
//   the next bracket is [t_{i*-1}, t_{i*+1}] (t_{-1} = lo, t_S = hi);
//   after R rounds: the largest Lambda seen (first seen on ties) and where.
//
// Mapping.  A block has four waves; NS waves (the node split) work on one
// interval, so a block covers 4 / NS intervals.  Each of the NS waves holds
// all S samples of the round (P = S / 64 rounded up to a power of two per
// lane, lanes beyond S duplicate the last sample and are masked) and sums
// over its 1/NS of the node table, node records arriving as wave-uniform
// scalar loads; the NS partial sums are added through LDS in wave order, so
// the result does not depend on timing.  The first wave of the interval
// finishes Lambda, finds (value, index) of the best sample with a butterfly
// over the wave, and publishes the next bracket through LDS.  Every wave
// runs exactly R rounds (groups past the last interval redo the last one
// and store nothing), so the block barriers are uniform.  Small node counts
// get NS = 4 to put enough waves on the chip; large ones NS = 1, which needs
// no LDS and no barrier.
//
// Sums use the simultaneous inversion of the evaluation kernels (group
// products of 8 differences, one reciprocal each).  When the weights
// alternate in sign the blocks of 16 nodes are summed by node pairs
// (pair_math.h), the Lebesgue sum from the block's even and odd sums; the
// blocks of the interval's two nodes, the same for every sample of the
// wave, and the blocks that failed the pair test are summed node by node in
// the loop (no masks), and the blocks far from the interval by octets (the
// block's eight even and eight odd nodes, each as one rational function;
// see "Octets" below).  A flagged
// sample (a hit
// on a node, which the zoom produces only once the bracket is below the
// spacing of binary64 numbers, or an extreme product) is recomputed with one
// division per pair and Lambda = 1 at a hit.
#include <cmath>

#include "fh_internal.h"
#include "pair_math.h"

namespace fhk {

namespace {

constexpr int kLmG = 8;  // nodes per simultaneous inversion

// t_i = lo + (i + 1) h, product and sum rounded separately
__device__ __forceinline__ double sample_at(double lo, double h, int i) {
#pragma clang fp contract(off)
  const double step = (double)(i + 1) * h;
  return lo + step;
}

// ---- Octets: the blocks far from the wave's interval ----
//
// The search takes the octets of pair_math.h (D only) for the blocks with at
// least kOctetGap whole blocks between them and the blocks of the wave's
// interval; the table uses them only if every block passed the octet test.
// Record per block: c, then for the even and the odd octet m, Q[0..7] and
// PD[0..7]; one spare.
constexpr int64_t kOctetRec = 36;

// The octet record of block b of the table (x, w: n nodes and weights);
// returns whether both octets passed (a block with no node below n passes).
__device__ bool octet_record(const double* __restrict__ x, const double* __restrict__ w,
                             int64_t n, int64_t b, double* __restrict__ rec) {
  const int64_t k0 = b * kPairBlock;
  const double c = pair_anchor(x, n, k0);
  rec[0] = c;
  rec[kOctetRec - 1] = 0.0;
  const bool e = octet_coefficients<false>(x, w, nullptr, n, k0, c, 0, rec + 1);
  const bool o = octet_coefficients<false>(x, w, nullptr, n, k0, c, 1, rec + 18);
  return (e && o) || k0 >= n;
}

// One workgroup: the octet records of the blocks [0, n_pad / 16) and
// *all_ok = 1 when every block passed.
__global__ void __launch_bounds__(256)
    k_pack_octets(const double* __restrict__ x, const double* __restrict__ w, int64_t n,
                  int64_t n_pad, double* __restrict__ oct, uint32_t* __restrict__ all_ok) {
  __shared__ int failed;
  if (threadIdx.x == 0) failed = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t b = threadIdx.x; b * kPairBlock < n_pad; b += blockDim.x)
    mine |= octet_record(x, w, n, b, oct + b * kOctetRec) ? 0 : 1;
  if (mine) atomicOr(&failed, 1);
  __syncthreads();
  if (threadIdx.x == 0) *all_ok = failed ? 0u : 1u;
}


// accumulate_f64_pairs for points that share their neighbouring nodes: all
// of the wave's points lie between the same two nodes, so the blocks that
// hold them, [near_lo, near_hi] (wave-uniform), are the same for every
// lane and are summed node by node right in the loop (groups of G,
// records through scalar loads, the Lebesgue sum from |w_k| |t_k|), and so
// are, with MIXED (some block of the table failed the pack's test), the
// blocks whose flag says they failed it.  With octets (wave-uniform: every
// block passed the octet test), the blocks below far_lo or above far_hi
// take their two octets' rational functions from oct (D and A only); every
// other block takes the pair sums with no mask.  Lane flags as in
// accumulate_f64.
template <int P, int G, bool R, bool L, bool MIXED>
__device__ __forceinline__ void accumulate_f64_pairs_known(
    const double (&xp)[P], const double* __restrict__ pr, const double* __restrict__ oct,
    const double* __restrict__ tx, const double* __restrict__ tw, const double* __restrict__ twf,
    int64_t k_begin, int64_t k_end, int32_t near_lo, int32_t near_hi, bool octets,
    int32_t far_lo, int32_t far_hi, double (&N)[P], double (&D)[P], double (&A)[P],
    bool (&bad)[P]) {
  static_assert((int)kPairBlock % G == 0, "blocks of whole node groups");
  const int b0 = (int)(k_begin / kPairBlock);
  const int nb = (int)((k_end - k_begin) / kPairBlock);
  for (int ib = 0; ib < nb; ++ib) {
    const int b = b0 + ib;
    if (!R && octets && (b < far_lo || b > far_hi)) {
      const double* __restrict__ o = oct + (int64_t)b * kOctetRec;
      const double c = o[0];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double x1 = xp[j] - c;
        double Qe, Pe, Qo, Po, unused;
        octet_eval<false>(o + 1, x1 - o[1], Qe, Pe, unused);
        octet_eval<false>(o + 18, x1 - o[18], Qo, Po, unused);
        // one reciprocal for both octets
        const double y = rcp_refined(Qe * Qo);
        const double E = Pe * (y * Qo), O = Po * (y * Qe);
        D[j] += E + O;
        if (L) A[j] += fabs(E - O);
      }
      continue;
    }
    const double* __restrict__ rec = pr + (int64_t)b * kPairRec;
    if ((b >= near_lo && b <= near_hi) || (MIXED && !pair_block_passed(rec))) {
      const double* __restrict__ px = tx + (int64_t)b * kPairBlock;
      const double* __restrict__ pw = tw + (int64_t)b * kPairBlock;
      const double* __restrict__ pv = twf + (int64_t)b * kPairBlock;
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
            if (R) N[j] = __builtin_fma(vk[i], t[i], N[j]);
            D[j] = __builtin_fma(wk[i], t[i], D[j]);
            if (L) A[j] = __builtin_fma(fabs(wk[i]), fabs(t[i]), A[j]);
          }
        }
      }
      continue;
    }
    double Nb[P], E[P], O[P], x1[P];
    const double c = rec[0];
#pragma unroll
    for (int j = 0; j < P; ++j) x1[j] = xp[j] - c;
    pair_group<P, R, false>(x1, rec + kPairHead, rec, Nb, E, true);
    __builtin_amdgcn_sched_barrier(0);
    pair_group<P, R, false>(x1, rec + kPairHead + 24, rec, Nb, O, false);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (R) N[j] += Nb[j];
      D[j] += E[j] + O[j];
      if (L) A[j] += fabs(E[j] - O[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) bad[j] |= !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
}

// (value, index) order of the search: larger value first, then smaller index
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

template <int P, int NS>
__global__ void __launch_bounds__(256)
    k_lebesgue_max(const double* __restrict__ tx, const double* __restrict__ tw,
                   const double* __restrict__ pr, const uint32_t* __restrict__ pok,
                   const double* __restrict__ oct, const uint32_t* __restrict__ oct_ok, int64_t n_pad,
                   int64_t n, int32_t samples, int32_t rounds, const uint32_t* __restrict__ alt,
                   double* __restrict__ lam_out, double* __restrict__ x_out) {
  constexpr int IG = 4 / NS;  // intervals per block
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int part = wave % NS, ig = wave / NS;
  const int64_t intervals = n - 1;
  const int64_t k_raw = (int64_t)blockIdx.x * IG + ig;
  const bool live = k_raw < intervals;
  const int64_t k = live ? k_raw : intervals - 1;

  // partial sums of waves 1..NS-1 (a token size when NS = 1: unused)
  constexpr int RW = NS > 1 ? NS - 1 : 1, RL = NS > 1 ? 64 * P : 1;
  __shared__ double red[IG][RW][2][RL];
  __shared__ int redbad[IG][RW][RL];
  __shared__ double brk[IG][2];

  const int64_t slice_len = n_pad / NS;
  const int64_t k_begin = part * slice_len, k_end = k_begin + slice_len;
  // sums by node pairs when the weights alternate in sign; every sample of
  // the wave lies in interval k, so the blocks of x_k and x_{k+1} are the
  // ones next to every sample (the loop runs over the padded table, whose
  // blocks beyond the nodes pass the test)
  const bool pairs = __builtin_amdgcn_readfirstlane(*alt) != 0;
  const bool mixed = pairs && !pair_table_ok(pok, n_pad);
  // octets for the blocks with kOctetGap whole blocks between them and the
  // interval's blocks, when every block of the table passed the octet test
  const bool octets = pairs && __builtin_amdgcn_readfirstlane(*oct_ok) != 0;
  const int32_t near_lo = (int32_t)(k / kPairBlock), near_hi = (int32_t)((k + 1) / kPairBlock);
  const int32_t far_lo = near_lo - kOctetGap, far_hi = near_hi + kOctetGap;

  double lo = tx[k], hi = tx[k + 1];
  double best = -INFINITY, best_x = NAN;
  for (int r = 0; r < rounds; ++r) {
    const double h = (hi - lo) / (double)(samples + 1);
    double xp[P], N[P], D[P], A[P];
    bool bad[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int i = j * 64 + lane;
      xp[j] = sample_at(lo, h, i < samples ? i : samples - 1);
      N[j] = 0.0;
      D[j] = 0.0;
      A[j] = 0.0;
      bad[j] = false;
    }
    if (mixed)
      accumulate_f64_pairs_known<P, kLmG, false, true, true>(
          xp, pr, oct, tx, tw, tw, k_begin, k_end, near_lo, near_hi, octets, far_lo, far_hi, N, D,
          A, bad);
    else if (pairs)
      accumulate_f64_pairs_known<P, kLmG, false, true, false>(
          xp, pr, oct, tx, tw, tw, k_begin, k_end, near_lo, near_hi, octets, far_lo, far_hi, N, D,
          A, bad);
    else
      accumulate_f64<P, kLmG, false, true>(xp, tx, tw, nullptr, k_begin, k_end, N, D, A, bad);

    if constexpr (NS > 1) {
      if (part > 0) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          red[ig][part - 1][0][j * 64 + lane] = D[j];
          red[ig][part - 1][1][j * 64 + lane] = A[j];
          redbad[ig][part - 1][j * 64 + lane] = bad[j];
        }
      }
      __syncthreads();
      if (part == 0) {
#pragma unroll
        for (int s = 0; s < NS - 1; ++s) {
#pragma unroll
          for (int j = 0; j < P; ++j) {
            D[j] += red[ig][s][0][j * 64 + lane];
            A[j] += red[ig][s][1][j * 64 + lane];
            bad[j] |= redbad[ig][s][j * 64 + lane] != 0;
          }
        }
      }
    }

    if (part == 0) {
      // Lambda at the lane's samples; the lane's best in ascending index
      double bv = -INFINITY;
      int bi = 0x7fffffff;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int i = j * 64 + lane;
        double v;
        if (bad[j]) {
          v = eval_point_exact<false, true>(xp[j], tx, tw, nullptr, n).l;
        } else {
          v = A[j] / fabs(D[j]);
        }
        if (i >= samples || v != v) v = -INFINITY;
        if (better(v, i, bv, bi)) {
          bv = v;
          bi = i;
        }
      }
      // butterfly over the wave: every lane ends with the wave's best
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (better(ov, oi, bv, bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (bv != -INFINITY) {  // some sample was a number
        if (bv > best) {
          best = bv;
          best_x = sample_at(lo, h, bi);
        }
        const double nlo = bi > 0 ? sample_at(lo, h, bi - 1) : lo;
        const double nhi = bi < samples - 1 ? sample_at(lo, h, bi + 1) : hi;
        lo = nlo;
        hi = nhi;
      }
      if constexpr (NS > 1) {
        if (lane == 0) {
          brk[ig][0] = lo;
          brk[ig][1] = hi;
        }
      }
    }
    if constexpr (NS > 1) {
      __syncthreads();
      lo = brk[ig][0];
      hi = brk[ig][1];
      // the partial-sum buffers are rewritten next round only after this barrier
    }
  }
  if (part == 0 && lane == 0 && live) {
    const bool found = best != -INFINITY;
    if (lam_out) lam_out[k] = found ? best : NAN;
    if (x_out) x_out[k] = found ? best_x : NAN;
  }
}

// The constant: the first largest interval value (NaN never counts), and
// where it is; a single node gives (1, x_0).  One block.
__global__ void __launch_bounds__(256)
    k_lebesgue_best(const double* __restrict__ lam, const double* __restrict__ xk,
                    int64_t intervals, const double* __restrict__ x0, double* __restrict__ best) {
  __shared__ double sv[4];
  __shared__ long long si[4];
  double bv = -INFINITY;
  long long bi = 0x7fffffffffffffffLL;
  for (int64_t i = threadIdx.x; i < intervals; i += 256) {
    const double v = lam[i];
    if (v > bv) {  // ascending per thread: the first of equal values stays
      bv = v;
      bi = i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const long long oi = __shfl_xor(bi, off, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[wave] = bv;
    si[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) {
        bv = sv[w];
        bi = si[w];
      }
    if (intervals == 0) {
      best[0] = 1.0;
      best[1] = x0[0];
    } else if (bv == -INFINITY) {
      best[0] = NAN;
      best[1] = NAN;
    } else {
      best[0] = bv;
      best[1] = xk[bi];
    }
  }
}

template <int P, int NS>
hipError_t launch_lm(const NodeTable& t, int64_t n, int32_t samples, int32_t rounds,
                     const uint32_t* alt, const LebesgueBufs& bufs, double* lam, double* xk,
                     hipStream_t s) {
  constexpr int IG = 4 / NS;
  const int64_t blocks = (n - 1 + IG - 1) / IG;
  k_lebesgue_max<P, NS><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
      t.x, t.w, t.pr, t.pok, bufs.oct, bufs.oct_ok, t.n_pad, n, samples, rounds, alt, lam, xk);
  return hipGetLastError();
}

template <int P>
hipError_t launch_lm_p(const NodeTable& t, int64_t n, int32_t samples, int32_t rounds,
                       const uint32_t* alt, const LebesgueBufs& bufs, double* lam, double* xk,
                       hipStream_t s) {
  const int64_t intervals = n - 1;
  // enough waves for the chip: about 4 per SIMD (1024 SIMDs)
  if (intervals >= 4096) return launch_lm<P, 1>(t, n, samples, rounds, alt, bufs, lam, xk, s);
  if (intervals >= 2048) return launch_lm<P, 2>(t, n, samples, rounds, alt, bufs, lam, xk, s);
  return launch_lm<P, 4>(t, n, samples, rounds, alt, bufs, lam, xk, s);
}

}  // namespace

size_t layout_lebesgue_max(void* ws, int64_t n, NodeTable* t, LebesgueBufs* bufs) {
  size_t off = layout_tables(ws, n, t);
  char* base = static_cast<char*>(ws);
  const size_t bytes = sizeof(double) * (size_t)(n > 1 ? n - 1 : 1);
  bufs->lam = base ? reinterpret_cast<double*>(base + off) : nullptr;
  off = align_up(off + bytes);
  bufs->xk = base ? reinterpret_cast<double*>(base + off) : nullptr;
  off = align_up(off + bytes);
  bufs->oct = base ? reinterpret_cast<double*>(base + off) : nullptr;
  off = align_up(off + sizeof(double) * (size_t)(t->n_pad / kPairBlock * kOctetRec));
  bufs->oct_ok = base ? reinterpret_cast<uint32_t*>(base + off) : nullptr;
  off = align_up(off + sizeof(uint32_t));
  return off;
}

hipError_t launch_lebesgue_max(const NodeTable& t, int64_t n, int32_t samples, int32_t rounds,
                               const uint32_t* alt, const LebesgueBufs& bufs, double* lam,
                               double* xk, double* best, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (n > 1) {
    k_pack_octets<<<dim3(1), dim3(256), 0, s>>>(t.x, t.w, n, t.n_pad, bufs.oct, bufs.oct_ok);
    e = hipGetLastError();
    const int p = (samples + 63) / 64;
    if (e != hipSuccess)
      return e;
    else if (p <= 1)
      e = launch_lm_p<1>(t, n, samples, rounds, alt, bufs, lam, xk, s);
    else if (p <= 2)
      e = launch_lm_p<2>(t, n, samples, rounds, alt, bufs, lam, xk, s);
    else if (p <= 4)
      e = launch_lm_p<4>(t, n, samples, rounds, alt, bufs, lam, xk, s);
    else
      e = launch_lm_p<8>(t, n, samples, rounds, alt, bufs, lam, xk, s);
  }
  if (e != hipSuccess || best == nullptr) return e;
  k_lebesgue_best<<<dim3(1), dim3(256), 0, s>>>(lam, xk, n - 1, t.x, best);
  return hipGetLastError();
}

}  // namespace fhk
