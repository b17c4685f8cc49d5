// Binary32 pair arithmetic of the precision-split kernels (single and
// batched): the LDS-staged node loop of one block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fhk {

constexpr int kTile = 32;     // binary32 partial-sum length (nodes)
constexpr int kStage = 256;   // records per LDS stage (= threads per block)

__device__ __forceinline__ bool not_finite32(float v) {
  return __builtin_amdgcn_classf(v, 0x207);  // NaN or +-inf
}

// |v| by clearing the sign bit with a VOP2 v_and_b32 against a mask held in
// a VGPR (an abs modifier, or an and with a known constant that the compiler
// folds into one, would force the slower VOP3 encoding).
__device__ __forceinline__ float abs_vop2(float v, uint32_t mask) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & mask);
}

// Sums of one block over the split node table s4[0, n_pad) (n_pad a multiple
// of 8): the block stages kStage records at a time in LDS (double
// buffered), every wave reads them back with uniform addresses, and each
// lane accumulates its P points in binary32 tile sums promoted to binary64
// every kTile nodes.  Must be called by all threads of the block.
template <int P, bool R, bool L>
__device__ __forceinline__ void split_block_sums(float4 (&stage)[2][kStage],
                                                 const float4* __restrict__ s4, int64_t n_pad,
                                                 uint32_t mask, const float (&xh)[P],
                                                 const float (&xl)[P], double (&N)[P],
                                                 double (&D)[P], double (&A)[P], bool (&bad)[P]) {
  const int tid = threadIdx.x;
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
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < P; ++j) t[q][j] = __builtin_amdgcn_rcpf(t[q][j]);
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

}  // namespace fhk
