// Octet launch variants of the binary64 evaluation: the octet records of
// the node tables and the points sorted by node block.
//
// The blocks far from a point take its octets (pair_math.h: each block's
// eight even and eight odd nodes as one rational function in monomial form,
// about a quarter fewer binary64 operations than node pairs).  A wave can
// use them without a per-lane choice only for blocks that serve every one of
// its points, so the launch first sorts the points by node block (a counting
// sort: per-tile histograms in LDS, one scan, a scatter with one reserved
// range per bin and tile), evaluates them in that order and writes each
// result to the point's original position.  Which form a block takes for a
// point depends only on the point and the table (the record's L and R), so
// the order of the points within a bin, which the atomics leave open, does
// not change any bit.
#include "fh_internal.h"
#include "pair_math.h"

namespace fhk {

namespace {

constexpr int kSortTile = 4096;    // points per workgroup of the sort
constexpr int kSortBinsMax = 4096;  // node blocks of a table the sort supports

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

__global__ void __launch_bounds__(256) k_sort_clear(int32_t* __restrict__ count, int32_t nb) {
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256) count[b] = 0;
}

__global__ void __launch_bounds__(256)
    k_sort_count(const double* __restrict__ x, int64_t m, const double* __restrict__ tx,
                 int32_t nb, int32_t* __restrict__ key, int32_t* __restrict__ count) {
  __shared__ int32_t lc[kSortBinsMax];
  for (int32_t b = threadIdx.x; b < nb; b += 256) lc[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int64_t end = base + kSortTile < m ? base + kSortTile : m;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) {
    const int32_t k = sort_key(x[i], tx, nb);
    key[i] = k;
    atomicAdd(&lc[k], 1);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < nb; b += 256)
    if (lc[b] != 0) atomicAdd(&count[b], lc[b]);
}

// one workgroup: cursor = exclusive prefix sums of count
__global__ void __launch_bounds__(256)
    k_sort_scan(const int32_t* __restrict__ count, int32_t nb, int32_t* __restrict__ cursor) {
  __shared__ int32_t part[256];
  const int32_t per = (nb + 255) / 256;
  const int32_t b0 = threadIdx.x * per;
  int32_t sum = 0;
  for (int32_t b = b0; b < b0 + per && b < nb; ++b) sum += count[b];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int t = 0; t < 256; ++t) {
      const int32_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t run = part[threadIdx.x];
  for (int32_t b = b0; b < b0 + per && b < nb; ++b) {
    cursor[b] = run;
    run += count[b];
  }
}

__global__ void __launch_bounds__(256)
    k_sort_scatter(const double* __restrict__ x, int64_t m, const int32_t* __restrict__ key,
                   int32_t nb, int32_t* __restrict__ cursor, double* __restrict__ xs,
                   int32_t* __restrict__ order) {
  constexpr int kPer = kSortTile / 256;
  __shared__ int32_t lc[kSortBinsMax];
  for (int32_t b = threadIdx.x; b < nb; b += 256) lc[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  int32_t k[kPer], rank[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = base + threadIdx.x + 256 * t;
    k[t] = i < m ? key[i] : -1;
    rank[t] = k[t] >= 0 ? atomicAdd(&lc[k[t]], 1) : 0;
  }
  __syncthreads();
  // one range per bin of this tile
  for (int32_t b = threadIdx.x; b < nb; b += 256)
    if (lc[b] != 0) lc[b] = atomicAdd(&cursor[b], lc[b]);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = base + threadIdx.x + 256 * t;
    if (k[t] < 0) continue;
    const int32_t pos = lc[k[t]] + rank[t];
    xs[pos] = x[i];
    order[pos] = (int32_t)i;
  }
}

// one workgroup per table: its octet records and summary word
__global__ void __launch_bounds__(256)
    k_octet_records(OctetTables a, int64_t n, int64_t n_pad) {
  const int c = blockIdx.x;
  __shared__ int failed;
  if (threadIdx.x == 0) failed = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t b = threadIdx.x; b * kPairBlock < n_pad; b += 256)
    mine |= octet_eval_record(a.x[c], a.w[c], a.wf[c], n, b, a.rec[c] + b * kOctetEvalRec) ? 0
                                                                                           : 1;
  if (mine) atomicOr(&failed, 1);
  __syncthreads();
  if (threadIdx.x == 0) *a.ok[c] = failed ? 0u : 1u;
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
  b->rec = reinterpret_cast<double*>(take(sizeof(double) * (size_t)(nb * kOctetEvalRec)));
  b->ok = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t)));
  b->count = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)nb));
  b->cursor = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)nb));
  b->key = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mm));
  b->xs = reinterpret_cast<double*>(take(sizeof(double) * (size_t)mm));
  b->order = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mm));
  return off;
}

hipError_t launch_octet_records(const OctetTables& a, int32_t K, int64_t n, int64_t n_pad,
                                hipStream_t s) {
  k_octet_records<<<dim3((unsigned)K), dim3(256), 0, s>>>(a, n, n_pad);
  return hipGetLastError();
}

hipError_t launch_sort_points(const double* x, int64_t m, const double* tx, int64_t n_pad,
                              const OctetBufs& b, hipStream_t s) {
  const int32_t nb = (int32_t)(n_pad / kPairBlock);
  const unsigned tiles = (unsigned)((m + kSortTile - 1) / kSortTile);
  k_sort_clear<<<dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s>>>(b.count, nb);
  k_sort_count<<<dim3(tiles), dim3(256), 0, s>>>(x, m, tx, nb, b.key, b.count);
  k_sort_scan<<<dim3(1), dim3(256), 0, s>>>(b.count, nb, b.cursor);
  k_sort_scatter<<<dim3(tiles), dim3(256), 0, s>>>(x, m, b.key, nb, b.cursor, b.xs, b.order);
  return hipGetLastError();
}

}  // namespace fhk
