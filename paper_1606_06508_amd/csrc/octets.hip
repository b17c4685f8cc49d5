// Octet launch variants of the binary64 evaluation: the octet records of
// the node tables and the points sorted by node block.
//
// The blocks far from a point take its octets (pair_math.h: each block's
// eight even and eight odd nodes as one rational function in monomial form,
// about a quarter fewer binary64 operations than node pairs).  A wave can
// use them without a per-lane choice only for blocks that serve every one of
// its points, so the launch first sorts the points by node block -- a
// counting sort in chunks of kChunkTiles tiles: per tile its counts per
// block (LDS), per chunk the sorted start of each tile's run of each block,
// then every point to its place -- evaluates them in that order and writes
// each result to the point's original position.  The points of a chunk
// keep the chunk's range of positions, so the results of a wave go to one
// chunk's stretch of each output array and its cache lines fill before
// they leave the L2.  Which form a block takes for a point depends only on
// the point and the table (the record's L and R), so the order of the
// points inside a run, which the LDS atomics leave open, changes no bit.
#include "fh_internal.h"
#include "pair_math.h"

namespace fhk {

namespace {

constexpr int kSortBinsMax = 4096;  // node blocks of a table the sort supports
constexpr int kChunkTiles = 64;     // tiles whose points stay together in sorted order

__device__ __forceinline__ int32_t sort_key(double v, const double* __restrict__ tx, int32_t nb) {
  // the last block whose first node lies below v (0 if none, or v NaN)
  int32_t lo = 0, hi = nb;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (tx[(int64_t)mid * kPairBlock] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo > 0 ? lo - 1 : 0;
}

// One workgroup per tile of `tile` points: each point's block into key and
// the tile's count per block into row blockIdx.x of hist.
__global__ void __launch_bounds__(256)
    k_sort_count(const double* __restrict__ x, int64_t m, int64_t tile,
                 const double* __restrict__ tx, int32_t nb, int32_t* __restrict__ key,
                 int32_t* __restrict__ hist) {
  __shared__ int32_t lc[kSortBinsMax];
  for (int32_t b = threadIdx.x; b < nb; b += 256) lc[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * tile;
  const int64_t end = base + tile < m ? base + tile : m;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) {
    const int32_t k = sort_key(x[i], tx, nb);
    key[i] = k;
    atomicAdd(&lc[k], 1);
  }
  __syncthreads();
  int32_t* __restrict__ row = hist + (int64_t)blockIdx.x * nb;
  for (int32_t b = threadIdx.x; b < nb; b += 256) row[b] = lc[b];
}

// One workgroup per chunk of kChunkTiles tiles (the chunk's points take the
// sorted positions from the chunk's first point on, ordered by block, then
// by tile): each tile's count per block becomes the sorted position of the
// tile's first point in that block.
__global__ void __launch_bounds__(256)
    k_sort_offsets(int32_t* __restrict__ hist, int64_t tiles, int64_t tile, int32_t nb) {
  constexpr int kPerMax = kSortBinsMax / 256;
  __shared__ int32_t part[256];
  const int64_t t0 = (int64_t)blockIdx.x * kChunkTiles;
  const int32_t nt = (int32_t)(t0 + kChunkTiles < tiles ? kChunkTiles : tiles - t0);
  const int32_t per = (nb + 255) / 256;  // blocks per thread, at most kPerMax
  const int32_t b0 = threadIdx.x * per;
  int32_t tot[kPerMax];
  int32_t sum = 0;
  for (int q = 0; q < kPerMax; ++q) {
    tot[q] = 0;
    const int32_t b = b0 + q;
    if (q >= per || b >= nb) continue;
    // the chunk's counts of block b, loaded together
    int32_t c[kChunkTiles];
#pragma unroll
    for (int t = 0; t < kChunkTiles; ++t) c[t] = t < nt ? hist[(t0 + t) * nb + b] : 0;
#pragma unroll
    for (int t = 0; t < kChunkTiles; ++t) tot[q] += c[t];
    sum += tot[q];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int32_t v = part[t];
      part[t] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int32_t start = (int32_t)(t0 * tile) + part[threadIdx.x];
  for (int q = 0; q < kPerMax; ++q) {
    const int32_t b = b0 + q;
    if (q >= per || b >= nb) continue;
    int32_t c[kChunkTiles];
#pragma unroll
    for (int t = 0; t < kChunkTiles; ++t) c[t] = t < nt ? hist[(t0 + t) * nb + b] : 0;
    int32_t run = start;
#pragma unroll
    for (int t = 0; t < kChunkTiles; ++t) {
      if (t < nt) hist[(t0 + t) * nb + b] = run;
      run += c[t];
    }
    start += tot[q];
  }
}

// One workgroup per tile: every point to its sorted position, the start of
// its tile's run of its block plus its rank there (LDS atomics: the order
// inside a run is left open, which changes no result).
__global__ void __launch_bounds__(256)
    k_sort_scatter(const double* __restrict__ x, int64_t m, int64_t tile,
                   const int32_t* __restrict__ key, const int32_t* __restrict__ off, int32_t nb,
                   double* __restrict__ xs, int32_t* __restrict__ order) {
  __shared__ int32_t lc[kSortBinsMax];
  const int32_t* __restrict__ row = off + (int64_t)blockIdx.x * nb;
  for (int32_t b = threadIdx.x; b < nb; b += 256) lc[b] = row[b];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * tile;
  const int64_t end = base + tile < m ? base + tile : m;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) {
    const int32_t pos = atomicAdd(&lc[key[i]], 1);
    xs[pos] = x[i];
    order[pos] = (int32_t)i;
  }
}

// Octet records: grid (groups of 128 blocks, tables), one thread per octet
// (2 per block); each table's summary word is set by k_octet_flags first
// and cleared by any octet that fails the test (a block with no node below
// n passes).
__global__ void __launch_bounds__(256) k_octet_flags(OctetTables a) {
  if (threadIdx.x == 0) *a.ok[blockIdx.x] = 1u;
}

__global__ void __launch_bounds__(256)
    k_octet_records(OctetTables a, int64_t n, int64_t n_pad) {
  const int c = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * 128 + (threadIdx.x >> 1);
  const int g = threadIdx.x & 1;
  if (b * kPairBlock >= n_pad) return;
  double* rec = a.rec[c] + b * kOctetEvalRec;
  const int64_t k0 = b * kPairBlock;
  const double c0 = pair_anchor(a.x[c], n, k0);
  if (g == 0) {
    const int64_t kl = k0 - 16 * kOctetGap - 1, kr = k0 + 16 * (kOctetGap + 1);
    rec[0] = c0;
    rec[51] = kl >= 0 && kl < n ? a.x[c][kl] : -__builtin_inf();
    rec[52] = kr < n ? a.x[c][kr] : __builtin_inf();
    rec[kOctetEvalRec - 1] = 0.0;
  }
  const bool ok = octet_coefficients<true>(a.x[c], a.w[c], a.wf[c], n, k0, c0, g,
                                           rec + 1 + 25 * g) ||
                  k0 >= n;
  if (!ok) atomicAnd(a.ok[c], 0u);
}

// Points per tile of the sort: 1024, doubled until the tiles' count rows
// take at most 2^24 entries.
static int64_t sort_tile(int64_t m, int64_t nb) {
  int64_t tile = 1024;
  while ((m + tile - 1) / tile * nb > (int64_t(1) << 24)) tile *= 2;
  return tile;
}

}  // namespace

bool octets_possible(int64_t n, int64_t m) {
  const int64_t nb = round_up(n, kNodePad) / kPairBlock;
  return n > 1 && nb <= kSortBinsMax && m >= 1 && m <= 0x7fffffffLL;
}

size_t layout_octets(void* ws, int64_t n, int64_t m, OctetBufs* b) {
  NodeTable t;
  size_t off = layout_tables(nullptr, n, &t);
  char* base = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const int64_t nb = t.n_pad / kPairBlock;
  const int64_t mm = m > 0 ? m : 0;
  const int64_t tiles = mm > 0 ? (mm + sort_tile(mm, nb) - 1) / sort_tile(mm, nb) : 0;
  b->rec = reinterpret_cast<double*>(take(sizeof(double) * (size_t)(nb * kOctetEvalRec)));
  b->ok = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t)));
  b->hist = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)(tiles * nb)));
  b->key = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mm));
  b->xs = reinterpret_cast<double*>(take(sizeof(double) * (size_t)mm));
  b->order = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mm));
  return off;
}

hipError_t launch_octet_records(const OctetTables& a, int32_t K, int64_t n, int64_t n_pad,
                                hipStream_t s) {
  const int64_t nb = n_pad / kPairBlock;
  k_octet_flags<<<dim3((unsigned)K), dim3(64), 0, s>>>(a);
  k_octet_records<<<dim3((unsigned)((nb + 127) / 128), (unsigned)K), dim3(256), 0, s>>>(a, n,
                                                                                       n_pad);
  return hipGetLastError();
}

hipError_t launch_sort_points(const double* x, int64_t m, const double* tx, int64_t n_pad,
                              const OctetBufs& b, hipStream_t s) {
  const int32_t nb = (int32_t)(n_pad / kPairBlock);
  const int64_t tile = sort_tile(m, nb);
  const int64_t tiles = (m + tile - 1) / tile;
  const unsigned chunks = (unsigned)((tiles + kChunkTiles - 1) / kChunkTiles);
  k_sort_count<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(x, m, tile, tx, nb, b.key, b.hist);
  k_sort_offsets<<<dim3(chunks), dim3(256), 0, s>>>(b.hist, tiles, tile, nb);
  k_sort_scatter<<<dim3((unsigned)tiles), dim3(256), 0, s>>>(x, m, tile, b.key, b.hist, nb, b.xs,
                                                             b.order);
  return hipGetLastError();
}

}  // namespace fhk
