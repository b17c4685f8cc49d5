// Weight pass and node-table packing (gfx950).
//
// Weights follow the barycentric form of Floater & Hormann (2007):
//   w_k = sum_{i in J_k} (-1)^i / prod_{j=i..i+d, j!=k} (x_k - x_j),
//   J_k = { max(0, k-d) <= i <= min(k, n-1-d) }.
// One thread per node, O(d^2) work each, reading the block's node window
// from LDS.  The products run in ascending j, each term is one IEEE
// division, and the terms are added in ascending i with FMA contraction
// disabled, so the weights are reproducible bit-for-bit on any IEEE machine
// that follows the same order.
#include "fh_internal.h"
#include "split_math.h"
#include "weight_math.h"

namespace fhk {

// LDS: the block's node window is staged in LDS first (d <= kWeightLdsMaxD).
template <bool LDS>
__global__ void __launch_bounds__(256) k_weights(const double* __restrict__ x, int64_t n, int32_t d,
                                                 double* __restrict__ w, uint32_t* status) {
  extern __shared__ double xs[];
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
  const int64_t k = base + threadIdx.x;
  if constexpr (LDS) stage_weight_window(x, n, d, base, xs);
  if (k >= n) return;
  uint32_t flags = node_checks(x, n, k);
  if constexpr (LDS)
    w[k] = node_weight_of([&](int64_t j) { return xs[j - base + d]; }, n, d, k, &flags);
  else
    w[k] = node_weight(x, n, d, k, &flags);
  if (flags) atomicOr(status, flags);
}

__global__ void k_set_word(uint32_t* p, uint32_t v) { *p = v; }

// Node-pair records of the binary64 pair variants (layout, construction
// and use in pair_math.h).  A table with a block that fails the pack's test
// is summed node by node (the pair variants check the summary words pok
// first).  One thread per pair (threads 0..7 of each group of 16) and one
// per header (thread 8, which returns whether the block passed or holds no
// node); w and v of the CUDA block's 256 records come from LDS (sw, swf).
__device__ bool pack_pair_records(const double* __restrict__ x, int64_t n, int64_t n_pad,
                                  int64_t base, const double* sw, const double* swf,
                                  double* __restrict__ pr) {
  const int tid = threadIdx.x, lb = tid >> 4, t16 = tid & 15;
  const int64_t b = (base >> 4) + lb, k0 = b * kPairBlock;
  if (t16 > 8) return false;
  if (k0 >= n_pad) return t16 == 8;
  double* __restrict__ rec = pr + b * kPairRec;
  const double* bw = sw + lb * 16;
  const double* bv = swf + lb * 16;
  if (t16 < 8) {
    pair_record_pair(x, n, k0, bw, bv, t16, rec);
    return false;
  }
  return pair_record_header(x, n, k0, bw, bv, rec);
}

// The pair records of the CUDA block's 16 node blocks and their summary
// word (one word per CUDA block, so no word has two writers).
__device__ __forceinline__ void pack_pairs_and_summary(const double* __restrict__ x, int64_t n,
                                                       int64_t n_pad, int64_t base,
                                                       const double* sw, const double* swf,
                                                       uint32_t* okw, double* __restrict__ pr,
                                                       uint32_t* __restrict__ pok) {
  if (pack_pair_records(x, n, n_pad, base, sw, swf, pr)) atomicOr(okw, 1u << (threadIdx.x >> 4));
  __syncthreads();
  if (threadIdx.x == 0) pok[blockIdx.x] = *okw;
}

// FP64 node table: x_k, w_k, w_k f_k (one rounding), padded with zero-weight
// copies of the last node.  w_in (if given) replaces the weight pass;
// values may be NULL (Lebesgue only) and then w f is stored as 0.
template <bool LDS>
__global__ void __launch_bounds__(256) k_pack(const double* __restrict__ x,
                                              const double* __restrict__ f,
                                              const double* __restrict__ w_in, int64_t n,
                                              int32_t d, int64_t n_pad, double* __restrict__ tx,
                                              double* __restrict__ tw, double* __restrict__ twf,
                                              double* __restrict__ tf,
                                              double* __restrict__ tpr,
                                              uint32_t* __restrict__ tpok, uint32_t* status) {
#pragma clang fp contract(off)
  extern __shared__ double xs[];
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
  const int64_t k = base + threadIdx.x;
  // status word 3 = 1 while the weights alternate in sign: always for the
  // library's weights (every term of w_k has the sign (-1)^(k-d)); caller
  // weights start at 1 (k_set_word, launched before) and any pair that does
  // not alternate strictly clears it
  if (k == 0 && w_in == nullptr) status[3] = 1u;
  if constexpr (LDS) stage_weight_window(x, n, d, base, xs);
  // every thread reaches the barrier before the pair records
  __shared__ double sw[256], swf[256];
  __shared__ uint32_t okw;
  double wk = 0.0, vk = 0.0;
  if (k < n) {
    uint32_t flags = node_checks(x, n, k);
    if constexpr (LDS) {
      wk = node_weight_of([&](int64_t j) { return xs[j - base + d]; }, n, d, k, &flags);
    } else if (w_in) {
      wk = w_in[k];
      if (k + 1 < n && !(wk * w_in[k + 1] < 0.0)) status[3] = 0u;
    } else {
      wk = node_weight(x, n, d, k, &flags);
    }
    vk = f ? wk * f[k] : 0.0;
    tx[k] = x[k];
    tw[k] = wk;
    twf[k] = vk;
    tf[k] = f ? f[k] : 0.0;
    if (flags) atomicOr(status, flags);
  } else if (k < n_pad) {
    tx[k] = x[n - 1];
    tw[k] = 0.0;
    twf[k] = 0.0;
    tf[k] = 0.0;
  }
  sw[threadIdx.x] = wk;
  swf[threadIdx.x] = vk;
  if (threadIdx.x == 0) okw = 0u;
  __syncthreads();
  pack_pairs_and_summary(x, n, n_pad, base, sw, swf, &okw, tpr, tpok);
}

// The FP64 node tables of K degrees of one interpolant in one launch
// (blockIdx.y = c packs degree a.d[c] into the tables of workspace c), with
// the per-node arithmetic of k_pack: the same tables, bit for bit.
template <bool LDS>
__global__ void __launch_bounds__(256) k_pack_many(const double* __restrict__ x,
                                                   const double* __restrict__ f, int64_t n,
                                                   int64_t n_pad, PackMany a) {
#pragma clang fp contract(off)
  extern __shared__ double xs[];
  const int c = blockIdx.y;
  const int32_t d = a.d[c];
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
  const int64_t k = base + threadIdx.x;
  if (k == 0) a.status[c][3] = 1u;  // the library's weights alternate in sign
  if constexpr (LDS) stage_weight_window(x, n, d, base, xs);
  double* __restrict__ tx = a.x[c];
  double* __restrict__ tw = a.w[c];
  double* __restrict__ twf = a.wf[c];
  double* __restrict__ tf = a.f[c];
  // every thread reaches the barrier before the pair records
  __shared__ double sw[256], swf[256];
  __shared__ uint32_t okw;
  double wk = 0.0, vk = 0.0;
  if (k < n) {
    uint32_t flags = node_checks(x, n, k);
    if constexpr (LDS)
      wk = node_weight_of([&](int64_t j) { return xs[j - base + d]; }, n, d, k, &flags);
    else
      wk = node_weight(x, n, d, k, &flags);
    vk = f ? wk * f[k] : 0.0;
    tx[k] = x[k];
    tw[k] = wk;
    twf[k] = vk;
    tf[k] = f ? f[k] : 0.0;
    if (flags) atomicOr(a.status[c], flags);
  } else if (k < n_pad) {
    tx[k] = x[n - 1];
    tw[k] = 0.0;
    twf[k] = 0.0;
    tf[k] = 0.0;
  }
  sw[threadIdx.x] = wk;
  swf[threadIdx.x] = vk;
  if (threadIdx.x == 0) okw = 0u;
  __syncthreads();
  pack_pairs_and_summary(x, n, n_pad, base, sw, swf, &okw, a.pr[c], a.pok[c]);
}

// Split (binary32) node table (split_table_scale / split_record).  Every
// block reduces the whole table itself (n is small next to the evaluation;
// doing it per block avoids a second pass and any atomics); block 0 stores
// e and ef - e in status words 1 and 2 and the table's conditioning flag
// (split_table_wide) in status word 4.
__global__ void __launch_bounds__(256) k_pack_split(const double* __restrict__ tx,
                                                    const double* __restrict__ tw,
                                                    const double* __restrict__ twf, int64_t n,
                                                    int64_t n_pad, float4* __restrict__ s4,
                                                    int32_t* scale_out) {
  __shared__ double red[4][256];
  const SplitScale sc = split_table_scale(tx, tw, twf, n, n_pad, red);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_pad)
    s4[k] = split_record(k < n ? tx[k] : split_pad_x(tx[0], tx[n - 1]), tw[k], twf[k], sc);
  if (blockIdx.x == 0) {
    // block 0 also decides whether the table is too ill-conditioned for
    // binary32 terms (status word 4)
    const int wide = split_table_wide(tx, tw, n, red);
    if (threadIdx.x == 0) {
      scale_out[0] = sc.e;
      scale_out[1] = sc.shift;
      scale_out[3] = wide;
    }
  }
}

size_t layout_tables(void* ws, int64_t n, NodeTable* t) {
  const int64_t n_pad = round_up(n, kNodePad);
  char* base = static_cast<char*>(ws);
  size_t off = kStatusBytes;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  t->n_pad = n_pad;
  t->x = reinterpret_cast<double*>(take(sizeof(double) * n_pad));
  t->w = reinterpret_cast<double*>(take(sizeof(double) * n_pad));
  t->wf = reinterpret_cast<double*>(take(sizeof(double) * n_pad));
  t->f = reinterpret_cast<double*>(take(sizeof(double) * n_pad));
  t->s = reinterpret_cast<float4*>(take(sizeof(float4) * n_pad));
  t->pr = reinterpret_cast<double*>(take(sizeof(double) * kPairRec * (n_pad / kPairBlock)));
  t->pok = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * ((n_pad + 255) / 256)));
  return off;
}

hipError_t launch_weights(const double* nodes, int64_t n, int32_t d, double* w_out,
                          uint32_t* status, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  if (d <= kWeightLdsMaxD)
    k_weights<true><<<dim3((unsigned)blocks), dim3(256), weight_window_bytes(d, 256), s>>>(
        nodes, n, d, w_out, status);
  else
    k_weights<false><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(nodes, n, d, w_out, status);
  return hipGetLastError();
}

hipError_t launch_pack(const double* nodes, const double* values, const double* w_in, int64_t n,
                       int32_t d, const NodeTable& t, bool split, uint32_t* status,
                       hipStream_t s) {
  const int64_t blocks = (t.n_pad + 255) / 256;
  if (w_in) {
    k_set_word<<<1, 1, 0, s>>>(status + 3, 1u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (w_in == nullptr && d <= kWeightLdsMaxD)
    k_pack<true><<<dim3((unsigned)blocks), dim3(256), weight_window_bytes(d, 256), s>>>(
        nodes, values, w_in, n, d, t.n_pad, t.x, t.w, t.wf, t.f, t.pr, t.pok, status);
  else
    k_pack<false><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(nodes, values, w_in, n, d, t.n_pad,
                                                               t.x, t.w, t.wf, t.f, t.pr, t.pok, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !split) return e;
  k_pack_split<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
      t.x, t.w, t.wf, n, t.n_pad, t.s, reinterpret_cast<int32_t*>(status) + 1);
  return hipGetLastError();
}

hipError_t launch_pack_many(const double* nodes, const double* values, int64_t n,
                            const PackMany& a, int32_t K, hipStream_t s) {
  const int64_t n_pad = round_up(n, kNodePad);
  const dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)K);
  int32_t dmax = 0;
  for (int32_t c = 0; c < K; ++c) dmax = a.d[c] > dmax ? a.d[c] : dmax;
  if (dmax <= kWeightLdsMaxD)
    k_pack_many<true><<<grid, dim3(256), weight_window_bytes(dmax, 256), s>>>(nodes, values, n,
                                                                             n_pad, a);
  else
    k_pack_many<false><<<grid, dim3(256), 0, s>>>(nodes, values, n, n_pad, a);
  return hipGetLastError();
}

}  // namespace fhk
