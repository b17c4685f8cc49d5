// Several Floater-Hormann interpolants on the same nodes and points, in one
// launch (gfx950): K columns, column c with its own degree d_c and values
// f^(c).  Every interpolant's sums need the same reciprocals
// t_k = 1 / (x - x_k) of the point-node pairs; computing them once for all
// columns divides their cost (a difference, the simultaneous inversion of
// eight differences per v_rcp_f64) by the number of
// columns, leaving the three fused multiply-adds per pair and column
// (N += (w f) t, D += w t, L += |w| |t|).  When every column has the same
// degree the weights are shared and so are D and L: one fused multiply-add
// per pair and column for N, two per pair for D and L (vector-valued data).
//
// Mapping.  One point per lane, four waves per block, one wave per 64
// points; the columns are processed in chunks of KC per launch row (grid.y,
// a compile-time chunk size), each chunk recomputing the reciprocals.  Node
// records are wave-uniform scalar loads (SGPR operands): x_k once per group
// of eight nodes, then w^(c) and (w f)^(c) per column.  Per pair and column the
// operations are those of the single-interpolant kernel with one point per
// lane, groups of eight and no node split (same inversion, same sums in the
// same order), so each column's r and Lambda equal that kernel's bits.
// Flagged points (a zero, subnormal, infinite or NaN group product: an exact
// hit, a NaN point, extreme coordinates) are recomputed per column with one
// division per pair and the exact-hit branch.
#include "fh_internal.h"
#include "pair_math.h"
#include "weight_math.h"

namespace fhk {

namespace {

constexpr int kMultiG = 8;

// Weight table of K columns: tw[cw][n_pad] (cw = c, or 0 when shared),
// twf[c][n_pad] = w^(c) f^(c), tf[c][n_pad] = f^(c); tx[n_pad] shared.
// LDS: each block first stages its column's node window (degree at most
// kWeightLdsMaxD, LDS sized for the largest degree of the launch).
template <bool LDS>
__global__ void __launch_bounds__(256)
    k_pack_multi(const double* __restrict__ x, const double* __restrict__ f, int64_t n,
                 MultiDegrees deg, int32_t K, bool shared, int64_t n_pad,
                 double* __restrict__ tx, double* __restrict__ tw, double* __restrict__ twf,
                 double* __restrict__ tf, uint32_t* status) {
#pragma clang fp contract(off)
  extern __shared__ double xs[];
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
  const int64_t k = base + threadIdx.x;
  const int c = blockIdx.y;  // 0 .. K_pad - 1; columns from K on are zero padding
  const int32_t dc = c < K ? deg.d[shared ? 0 : c] : 0;
  if constexpr (LDS) stage_weight_window(x, n, dc, base, xs);
  if (k >= n_pad) return;
  double* w_c = tw + (shared ? 0 : (int64_t)c * n_pad);
  if (k >= n || c >= K) {
    if (c == 0) tx[k] = x[n - 1];
    if (c == 0 || !shared) w_c[k] = 0.0;
    twf[(int64_t)c * n_pad + k] = 0.0;
    tf[(int64_t)c * n_pad + k] = 0.0;
    return;
  }
  uint32_t flags = 0;
  double wk;
  // with shared weights each column recomputes them (O(d^2) per node)
  if constexpr (LDS)
    wk = node_weight_of([&](int64_t j) { return xs[j - base + dc]; }, n, dc, k, &flags);
  else
    wk = node_weight(x, n, dc, k, &flags);
  if (c == 0 || !shared) w_c[k] = wk;
  if (c == 0) {
    flags |= node_checks(x, n, k);
    tx[k] = x[k];
  }
  const double fk = f[(int64_t)c * n + k];
  twf[(int64_t)c * n_pad + k] = wk * fk;
  tf[(int64_t)c * n_pad + k] = fk;
  if (flags) atomicOr(status, flags);
}

// KC columns per launch row, a compile-time count: the column loop is
// straight-line code, so the scalar loads of one column's records overlap
// the previous column's arithmetic.  Columns past K read the zero padding
// of the tables and are not stored.
template <int KC, bool L, bool SH>
__global__ void __launch_bounds__(256)
    k_eval_multi(const double* __restrict__ x, int64_t m, const double* __restrict__ tx,
                 const double* __restrict__ tw, const double* __restrict__ twf,
                 const double* __restrict__ tf, int64_t n_pad, int64_t n, int32_t K,
                 double* __restrict__ r, double* __restrict__ lam) {
  const int lane = threadIdx.x & 63;
  const int c0 = blockIdx.y * KC;
  const int kc = K - c0 < KC ? K - c0 : KC;  // columns of this chunk that are stored
  const int64_t idx = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64 + lane;
  const double xp = x[idx < m ? idx : m - 1];
  constexpr int KD = SH ? 1 : KC;  // D and L sums per point
  double N[KC], D[KD], A[KD];
#pragma unroll
  for (int c = 0; c < KC; ++c) N[c] = 0.0;
#pragma unroll
  for (int c = 0; c < KD; ++c) D[c] = A[c] = 0.0;
  const int cnt = (int)n_pad;
  for (int k = 0; k < cnt; k += kMultiG) {
    double dl[kMultiG], t[kMultiG];
#pragma unroll
    for (int i = 0; i < kMultiG; ++i) dl[i] = xp - tx[k + i];
    group_product_reciprocals<kMultiG>(dl, t);
    if constexpr (SH) {
#pragma unroll
      for (int i = 0; i < kMultiG; ++i) {
        const double wk = tw[k + i];
        D[0] = __builtin_fma(wk, t[i], D[0]);
        if (L) A[0] = __builtin_fma(fabs(wk), fabs(t[i]), A[0]);
      }
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const double* __restrict__ pv = twf + (int64_t)(c0 + c) * n_pad + k;
      if constexpr (SH) {
#pragma unroll
        for (int i = 0; i < kMultiG; ++i) N[c] = __builtin_fma(pv[i], t[i], N[c]);
      } else {
        const double* __restrict__ pw = tw + (int64_t)(c0 + c) * n_pad + k;
#pragma unroll
        for (int i = 0; i < kMultiG; ++i) {
          D[c] = __builtin_fma(pw[i], t[i], D[c]);
          N[c] = __builtin_fma(pv[i], t[i], N[c]);
          if (L) A[c] = __builtin_fma(fabs(pw[i]), fabs(t[i]), A[c]);
        }
      }
    }
  }
  if (idx >= m) return;
  // a column's lane is flagged as in k_eval_f64: D not finite (a zero,
  // infinite or NaN group product makes every t NaN)
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    if (c >= kc) break;
    const int cd = SH ? 0 : c;
    const int64_t col = c0 + c;
    double rv, lv;
    if (!(fabs(D[cd]) <= 0x1.fffffffffffffp+1023)) {
      const PointRL e =
          eval_point_exact<true, L>(xp, tx, tw + (SH ? 0 : col * n_pad), tf + col * n_pad, n);
      rv = e.r;
      lv = e.l;
    } else {
      rv = N[c] / D[cd];
      lv = A[cd] / fabs(D[cd]);
    }
    r[col * m + idx] = rv;
    if (L) lam[col * m + idx] = lv;
  }
}

template <int KC, bool SH>
hipError_t launch_multi_kc(const double* x, int64_t m, const MultiTable& t, int64_t n, int32_t K,
                           double* r, double* lam, hipStream_t s) {
  const dim3 grid((unsigned)((m + 255) / 256), (unsigned)((K + KC - 1) / KC)), block(256);
  if (lam)
    k_eval_multi<KC, true, SH><<<grid, block, 0, s>>>(x, m, t.x, t.w, t.wf, t.f, t.n_pad, n, K,
                                                      r, lam);
  else
    k_eval_multi<KC, false, SH><<<grid, block, 0, s>>>(x, m, t.x, t.w, t.wf, t.f, t.n_pad, n, K,
                                                       r, lam);
  return hipGetLastError();
}

}  // namespace

size_t layout_multi(void* ws, int64_t n, int32_t K, MultiTable* t) {
  const int64_t n_pad = round_up(n, kNodePad);
  char* base = static_cast<char*>(ws);
  size_t off = kStatusBytes;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return reinterpret_cast<double*>(p);
  };
  t->n_pad = n_pad;
  t->x = take(sizeof(double) * n_pad);
  const int64_t kp = multi_padded_columns(K);
  t->w = take(sizeof(double) * n_pad * kp);
  t->wf = take(sizeof(double) * n_pad * kp);
  t->f = take(sizeof(double) * n_pad * kp);
  return off;
}

// Column chunking: at most 6 columns per launch row (8 with shared
// weights), balanced, rounded up to a compiled chunk size.  Measured on the
// sines workload: the d = 0..8 sweep runs 1.38 ms in chunks of 5 and
// 1.43 ms in one chunk of 9, where the record loads of nine columns exhaust
// the scalar registers; 16 value columns with shared weights take 0.83 ms
// in chunks of 8, 1.06 ms in chunks of 6 or 1.10 ms in one chunk of 16
// (whose scalar loads are then waited for in small batches).
static int multi_chunk(int32_t K, bool shared) {
  static const int sizes[] = {1, 2, 3, 4, 5, 6, 8};
  const int kmax = shared ? 8 : 6;
  const int chunks = (K + kmax - 1) / kmax;
  const int kc = (K + chunks - 1) / chunks;
  for (int v : sizes)
    if (v >= kc) return v;
  return 8;
}

// the chunks cover rows * kc < K + 8 columns
int64_t multi_padded_columns(int32_t K) { return (int64_t)K + 8; }

hipError_t launch_multi(const double* nodes, const double* values, int64_t n,
                        const MultiDegrees& deg, int32_t K, bool shared, const double* x,
                        int64_t m, const MultiTable& t, double* r, double* lam, uint32_t* status,
                        hipStream_t s) {
  const int kc = multi_chunk(K, shared);
  const int rows = (K + kc - 1) / kc;
  const dim3 pg((unsigned)((t.n_pad + 255) / 256), (unsigned)(rows * kc));
  int32_t dmax = 0;
  for (int32_t c = 0; c < K; ++c) dmax = deg.d[c] > dmax ? deg.d[c] : dmax;
  if (dmax <= kWeightLdsMaxD)
    k_pack_multi<true><<<pg, 256, weight_window_bytes(dmax, 256), s>>>(
        nodes, values, n, deg, K, shared, t.n_pad, t.x, t.w, t.wf, t.f, status);
  else
    k_pack_multi<false><<<pg, 256, 0, s>>>(nodes, values, n, deg, K, shared, t.n_pad, t.x, t.w,
                                           t.wf, t.f, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || m == 0) return e;
  switch (kc * 2 + (shared ? 1 : 0)) {
#define FH_MULTI_CASE(KC)                                                            \
  case KC * 2: return launch_multi_kc<KC, false>(x, m, t, n, K, r, lam, s);          \
  case KC * 2 + 1: return launch_multi_kc<KC, true>(x, m, t, n, K, r, lam, s);
    FH_MULTI_CASE(1) FH_MULTI_CASE(2) FH_MULTI_CASE(3) FH_MULTI_CASE(4) FH_MULTI_CASE(5)
    FH_MULTI_CASE(6) FH_MULTI_CASE(8)
#undef FH_MULTI_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fhk
