// Floater-Hormann weight of one node and the node-table checks, shared by
// the single-interpolant and batched packing kernels.
//   w_k = sum_{i in J_k} (-1)^i / prod_{j=i..i+d, j!=k} (x_k - x_j),
//   J_k = { max(0, k-d) <= i <= min(k, n-1-d) }   (Floater & Hormann 2007).
#pragma once

#include <hip/hip_runtime.h>

#include "fh.h"

namespace fhk {

// Weight of node k; ORs FH_FLAG_* into *flags.  xj(j) returns node j (from
// global memory or from a block's LDS copy: the arithmetic is the same).
template <class XJ>
__device__ inline double node_weight_of(XJ xj, int64_t n, int32_t d, int64_t k, uint32_t* flags) {
#pragma clang fp contract(off)
  const double xk = xj(k);
  const int64_t ilo = k - d > 0 ? k - d : 0;
  const int64_t ihi = k < n - 1 - d ? k : n - 1 - d;
  double s = 0.0;
  for (int64_t i = ilo; i <= ihi; ++i) {
    double prod = 1.0;
#pragma unroll 4
    for (int64_t j = i; j <= i + d; ++j)
      if (j != k) prod = prod * (xk - xj(j));
    // a zero, subnormal, infinite or NaN product means the weight cannot be
    // represented accurately
    if (!__builtin_isnormal(prod)) *flags |= FH_FLAG_RANGE;
    double term = 1.0 / prod;
    if (i & 1) term = -term;
    s = s + term;
  }
  return s;
}

__device__ inline double node_weight(const double* __restrict__ x, int64_t n, int32_t d, int64_t k,
                                     uint32_t* flags) {
  return node_weight_of([x](int64_t j) { return x[j]; }, n, d, k, flags);
}

// The nodes a block of B threads (nodes base .. base+B-1) needs for its
// weights: x[base-d .. base+B-1+d], copied to LDS with coalesced loads
// (entries outside 0..n-1 are never read and left unset).  Every thread of
// the block must call it.  A weight then reads LDS instead of making
// (d+1)^2 dependent trips to L2.
constexpr int32_t kWeightLdsMaxD = 3968;  // (256 + 2 d) doubles <= 64 KiB

__device__ inline void stage_weight_window(const double* __restrict__ x, int64_t n, int32_t d,
                                           int64_t base, double* xs) {
  const int64_t lo = base - d;
  const int64_t cnt = (int64_t)blockDim.x + 2 * (int64_t)d;
  for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int64_t j = lo + t;
    if (j >= 0 && j < n) xs[t] = x[j];
  }
  __syncthreads();
}

inline size_t weight_window_bytes(int32_t d, int block) {
  return sizeof(double) * ((size_t)block + 2 * (size_t)d);
}

__device__ inline uint32_t node_checks(const double* __restrict__ x, int64_t n, int64_t k) {
  uint32_t f = 0;
  const double xk = x[k];
  if (!__builtin_isfinite(xk)) f |= FH_FLAG_NONFINITE;
  if (k + 1 < n && !(xk < x[k + 1])) f |= FH_FLAG_NODES;
  return f;
}

}  // namespace fhk
