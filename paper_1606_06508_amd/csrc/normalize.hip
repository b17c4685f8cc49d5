// Batched vector and quaternion normalization (gfx950): the scaling
// algorithms of Mascarenhas, "Fast and accurate normalization of vectors
// and quaternions" (Scale2D / Scale3D of Section 2, Normalize2D /
// Normalize3D of Section 3, Normalize4D of Section 4, parameters of
// Table 2), the two quotient algorithms of the Introduction and the naive
// formula.
//
// The work per vector is a handful of compares, one scaling multiply, a
// sum of squares, one square root and one division, against 20 to 72 bytes
// of HBM traffic: the kernels are bound by HBM bandwidth.  Lanes take
// consecutive vectors (grid-stride), so the loads of a wave cover one
// contiguous span (array-of-structs) or are unit stride (struct-of-arrays);
// aligned array-of-structs data move in 16-byte loads and stores, several
// vectors per lane where one vector is not a whole number of 16 bytes.
//
// Scaling is branch-free: the largest magnitude m comes from each
// procedure's comparison tree, then every entry is multiplied by
// s in {1, sigma_max, sigma_min} (a power of two, so the product is exact;
// multiplying by 1 gives the unscaled entry bit for bit), and the result
// length is r~ times 1/s.  Sums of squares run left to right with FMA
// contraction off; sqrt and 1/r~ are the correctly rounded IEEE operations
// of the working precision.  The zero exits of the trees are taken only
// when no entry compared with "<" alone is NaN, so NaN input always gives
// NaN output (the NaN statement of Section 2).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nrm.h"

namespace nrmk {

// Table 2: tau_min, sigma_min, tau_max, sigma_max and the inverse scales.
template <typename T>
struct Table2;
template <>
struct Table2<float> {
  static constexpr float tmin = 0x1p-49f, smin = 0x1p100f, tmax = 0x1p62f, smax = 0x1p-66f;
  static constexpr float inv_smin = 0x1p-100f, inv_smax = 0x1p66f;
};
template <>
struct Table2<double> {
  static constexpr double tmin = 0x1p-482, smin = 0x1p592, tmax = 0x1p510, smax = 0x1p-514;
  static constexpr double inv_smin = 0x1p-592, inv_smax = 0x1p514;
};

template <typename T>
__device__ __forceinline__ T mag(T v) {
  return __builtin_fabs(v);
}
template <>
__device__ __forceinline__ float mag<float>(float v) {
  return __builtin_fabsf(v);
}

template <typename T>
__device__ __forceinline__ T sqrt_cr(T v) {
  return __builtin_sqrt(v);
}
template <>
__device__ __forceinline__ float sqrt_cr<float>(float v) {
  return __builtin_sqrtf(v);
}

// Largest magnitude by the comparison tree of Scale2D / Scale3D /
// Normalize4D; *zero is set when the tree's zero exit is taken.
template <typename T>
__device__ __forceinline__ T tree_max(const T (&x)[2], bool* zero) {
  T m = mag(x[0]);
  const bool ge = m >= mag(x[1]);
  *zero = ge && m == T(0);
  return ge ? m : mag(x[1]);
}
template <typename T>
__device__ __forceinline__ T tree_max(const T (&x)[3], bool* zero) {
  const T a0 = mag(x[0]), a1 = mag(x[1]), a2 = mag(x[2]);
  T m = a0;
  *zero = false;
  if (m < a1) {
    m = a1;
    if (m < a2) m = a2;
  } else if (m >= a2) {
    *zero = m == T(0) && x[1] == x[1];
  } else {
    m = a2;
  }
  return m;
}
template <typename T>
__device__ __forceinline__ T tree_max(const T (&x)[4], bool* zero) {
  const T a0 = mag(x[0]), a1 = mag(x[1]), a2 = mag(x[2]), a3 = mag(x[3]);
  T m = a0;
  *zero = false;
  if (m < a1) {
    m = a1;
    if (m < a2) m = a2;
    if (m < a3) m = a3;
  } else if (m < a2) {
    m = a2;
    if (m < a3) m = a3;
  } else if (m >= a3) {
    *zero = m == T(0) && x[1] == x[1] && x[2] == x[2];
  } else {
    m = a3;
  }
  return m;
}

template <typename T, int N>
__device__ __forceinline__ T sum_squares(const T (&y)[N]) {
#pragma clang fp contract(off)
  T acc = y[0] * y[0];
#pragma unroll
  for (int k = 1; k < N; ++k) acc = acc + y[k] * y[k];
  return acc;
}

// Normalize2D / Normalize3D / Normalize4D.
template <typename T, int N>
__device__ __forceinline__ void scaling(const T (&x)[N], T* r, T (&xh)[N]) {
#pragma clang fp contract(off)
  using P = Table2<T>;
  bool zero;
  const T m = tree_max(x, &zero);
  if (zero) {
    *r = T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) xh[k] = (N == 4 && k == 2) ? T(1) : T(0);
    return;
  }
  const bool low = !(m >= P::tmin), high = !low && !(m <= P::tmax);
  const T s = low ? P::smin : (high ? P::smax : T(1));
  const T inv = low ? P::inv_smin : (high ? P::inv_smax : T(1));
  T y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) y[k] = s * x[k];
  const T rt = sqrt_cr(sum_squares(y));
  const T h = T(1) / rt;
  *r = inv * rt;
#pragma unroll
  for (int k = 0; k < N; ++k) xh[k] = h * y[k];
}

// Algorithm 1: divide by the largest magnitude.
template <typename T, int N>
__device__ __forceinline__ void quotient(const T (&x)[N], T* r, T (&xh)[N]) {
#pragma clang fp contract(off)
  T m = mag(x[0]);
#pragma unroll
  for (int k = 1; k < N; ++k)
    if (mag(x[k]) > m) m = mag(x[k]);
  if (m == T(0)) {
    *r = T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) xh[k] = x[k];
    return;
  }
  T y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) y[k] = x[k] / m;
  const T sq = sqrt_cr(sum_squares(y));
  *r = m * sq;
#pragma unroll
  for (int k = 0; k < N; ++k) xh[k] = y[k] / sq;
}

// Algorithm 2 (three dimensions): divide by the largest entry x_p.
template <typename T>
__device__ __forceinline__ void quotient_pivot(const T (&x)[3], T* r, T (&xh)[3]) {
#pragma clang fp contract(off)
  int p;
  if (mag(x[0]) > mag(x[1])) {
    p = mag(x[2]) > mag(x[0]) ? 2 : 0;
  } else if (mag(x[2]) >= mag(x[1])) {
    if (x[2] == T(0)) {
      *r = T(0);
      xh[0] = xh[1] = xh[2] = T(0);
      return;
    }
    p = 2;
  } else {
    p = 1;
  }
  const int a = p == 0 ? 1 : 0, b = p == 2 ? 1 : 2;
  const T xp = x[p];
  const T qa = x[a] / xp, qb = x[b] / xp;
  const T h = sqrt_cr(T(1) + qa * qa + qb * qb);
  *r = mag(xp) * h;
  const T sp = __builtin_copysign(T(1), xp) / h;
  xh[a] = qa * sp;
  xh[b] = qb * sp;
  xh[p] = sp;
}

template <typename T, int N>
__device__ __forceinline__ void naive(const T (&x)[N], T* r, T (&xh)[N]) {
#pragma clang fp contract(off)
  const T rt = sqrt_cr(sum_squares(x));
  const T h = T(1) / rt;
  *r = rt;
#pragma unroll
  for (int k = 0; k < N; ++k) xh[k] = h * x[k];
}

template <typename T, int N, int METHOD>
__device__ __forceinline__ void normalize_one(const T (&v)[N], T* len, T (&o)[N]) {
  if constexpr (METHOD == NRM_SCALING) {
    scaling(v, len, o);
  } else if constexpr (METHOD == NRM_QUOTIENT) {
    quotient(v, len, o);
  } else if constexpr (METHOD == NRM_QUOTIENT_PIVOT) {
    if constexpr (N == 3) quotient_pivot(v, len, o);
  } else {
    naive(v, len, o);
  }
}

// One vector per lane and step; any alignment.
template <typename T, int N, int LAYOUT, int METHOD>
__global__ void __launch_bounds__(256)
    k_normalize(const T* __restrict__ x, int64_t n, T* __restrict__ r, T* __restrict__ xh) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    T v[N], o[N], len;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = LAYOUT == NRM_AOS ? x[i * N + k] : x[k * n + i];
    normalize_one<T, N, METHOD>(v, &len, o);
    if (r) r[i] = len;
    if (xh) {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (LAYOUT == NRM_AOS)
          xh[i * N + k] = o[k];
        else
          xh[k * n + i] = o[k];
      }
    }
  }
}

// Array-of-structs with 16-byte aligned arrays: each lane takes V
// consecutive vectors, V N sizeof(T) a multiple of 16 bytes, and moves them
// with 16-byte loads and stores (the lengths with V-wide stores when
// V sizeof(T) is 8 or 16 bytes).  The lanes of a wave cover one contiguous
// span per step.  The tail (n mod V vectors) is left to k_normalize.
template <typename T, int N, int METHOD, int V>
__global__ void __launch_bounds__(256)
    k_normalize_aos_vec(const T* __restrict__ x, int64_t groups, T* __restrict__ r,
                        T* __restrict__ xh) {
  constexpr int kChunks = V * N * (int)sizeof(T) / 16;
  static_assert(V * N * sizeof(T) % 16 == 0, "whole 16-byte chunks");
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < groups; gi += stride) {
    union {
      uint4 c[kChunks];
      T e[V * N];
    } in, out;
    const uint4* src = reinterpret_cast<const uint4*>(x) + gi * kChunks;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) in.c[c] = src[c];
    T len[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      T v[N], o[N];
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] = in.e[j * N + k];
      normalize_one<T, N, METHOD>(v, &len[j], o);
#pragma unroll
      for (int k = 0; k < N; ++k) out.e[j * N + k] = o[k];
    }
    if (xh) {
      uint4* dst = reinterpret_cast<uint4*>(xh) + gi * kChunks;
#pragma unroll
      for (int c = 0; c < kChunks; ++c) dst[c] = out.c[c];
    }
    if (r) {
#pragma unroll
      for (int j = 0; j < V; ++j) r[gi * V + j] = len[j];
    }
  }
}

static int64_t grid_for(int64_t items) {
  int64_t blocks = (items + 255) / 256;
  return blocks > 65536 ? 65536 : (blocks < 1 ? 1 : blocks);  // grid-stride beyond
}

// Vectors per lane of the 16-byte path: the least V with V N sizeof(T) a
// multiple of 16.
template <typename T, int N>
constexpr int vec_group() {
  return (N * sizeof(T)) % 16 == 0 ? 1 : ((2 * N * sizeof(T)) % 16 == 0 ? 2 : 4);
}

template <typename T, int N, int LAYOUT, int METHOD>
static void launch_method(const T* x, int64_t n, T* r, T* xh, bool aligned, hipStream_t s) {
  const dim3 block(256);
  int64_t done = 0;
  if constexpr (LAYOUT == NRM_AOS) {
    constexpr int V = vec_group<T, N>();
    const int64_t groups = n / V;
    if (aligned && groups > 0) {
      k_normalize_aos_vec<T, N, METHOD, V>
          <<<dim3((unsigned)grid_for(groups)), block, 0, s>>>(x, groups, r, xh);
      done = groups * V;
    }
  }
  if (done < n) {
    // the remaining vectors (all of them on the generic path)
    const int64_t rest = n - done;
    if (LAYOUT == NRM_AOS)
      k_normalize<T, N, LAYOUT, METHOD><<<dim3((unsigned)grid_for(rest)), block, 0, s>>>(
          x + done * N, rest, r ? r + done : nullptr, xh ? xh + done * N : nullptr);
    else
      k_normalize<T, N, LAYOUT, METHOD><<<dim3((unsigned)grid_for(n)), block, 0, s>>>(x, n, r,
                                                                                      xh);
  }
}

template <typename T, int N, int LAYOUT>
static hipError_t launch_layout(const T* x, int64_t n, T* r, T* xh, int method, bool aligned,
                                hipStream_t s) {
  switch (method) {
    case NRM_SCALING:
      launch_method<T, N, LAYOUT, NRM_SCALING>(x, n, r, xh, aligned, s);
      break;
    case NRM_QUOTIENT:
      launch_method<T, N, LAYOUT, NRM_QUOTIENT>(x, n, r, xh, aligned, s);
      break;
    case NRM_QUOTIENT_PIVOT:
      if constexpr (N == 3) {
        launch_method<T, N, LAYOUT, NRM_QUOTIENT_PIVOT>(x, n, r, xh, aligned, s);
        break;
      }
      return hipErrorInvalidValue;
    default:
      launch_method<T, N, LAYOUT, NRM_NAIVE>(x, n, r, xh, aligned, s);
      break;
  }
  return hipGetLastError();
}

template <typename T, int N>
static fh_status normalize(const T* x, int64_t n, T* r, T* xh, int32_t layout, int32_t method,
                           void* stream) {
  if (n < 0 || layout < NRM_AOS || layout > NRM_SOA) return FH_E_ARG;
  if (method < NRM_SCALING || method > NRM_NAIVE) return FH_E_ARG;
  if (method == NRM_QUOTIENT_PIVOT && N != 3) return FH_E_ARG;
  if (n == 0) return FH_OK;
  if (x == nullptr || (r == nullptr && xh == nullptr)) return FH_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the 16-byte path needs x and x_hat 16-byte aligned, and r aligned to
  // the width of its V-wide stores
  auto al = [](const void* p, uintptr_t a) { return p == nullptr || (uintptr_t)p % a == 0; };
  const bool aligned = al(x, 16) && al(xh, 16) && al(r, sizeof(T));
  const hipError_t e =
      layout == NRM_AOS ? launch_layout<T, N, NRM_AOS>(x, n, r, xh, method, aligned, s)
                        : launch_layout<T, N, NRM_SOA>(x, n, r, xh, method, aligned, s);
  return e == hipSuccess ? FH_OK : FH_E_HIP;
}

}  // namespace nrmk

extern "C" {

#define NRM_ENTRY(DIM, SFX, T)                                                                \
  fh_status nrm_normalize##DIM##_##SFX(const T* x, int64_t n, T* r_out, T* xhat_out,          \
                                        int32_t layout, int32_t method, void* stream) {       \
    return nrmk::normalize<T, DIM>(x, n, r_out, xhat_out, layout, method, stream);            \
  }
NRM_ENTRY(2, f32, float)
NRM_ENTRY(3, f32, float)
NRM_ENTRY(4, f32, float)
NRM_ENTRY(2, f64, double)
NRM_ENTRY(3, f64, double)
NRM_ENTRY(4, f64, double)
#undef NRM_ENTRY

}  // extern "C"
