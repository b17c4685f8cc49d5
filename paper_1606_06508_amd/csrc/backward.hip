// Adjoint of L = sum_p g_p r(x_p) (gfx950, binary64).
//
// With a_pk = w_k t_pk, t_pk = 1/(x_p - x_k), D_p = sum_k a_pk, r_p = N_p/D_p
// and c_p = g_p / D_p, the derivatives at non-hit points are
//   dL/dx_p   = c_p (r_p E_p - F_p),       E_p = sum_k w_k t_pk^2,
//                                          F_p = sum_k w_k f_k t_pk^2,
//   dL/df_k   = w_k S1_k,                  S1_k = sum_p c_p t_pk,
//   dL/dw_k   = f_k S1_k - S2_k,           S2_k = sum_p c_p r_p t_pk,
//   dL/dx_k|w = w_k (f_k S3_k - S4_k),     S3_k = sum_p c_p t_pk^2,
//                                          S4_k = sum_p c_p r_p t_pk^2,
// (differentiating the barycentric form of Floater & Hormann 2007 with
// respect to f_k, x_p, w_k and x_k).  At a hit x_p == x_j, r = f_j whatever
// the weights, so dL/df_j gets g_p, dL/dx_p = g_p r'(x_j) with the node
// formula r'(x_j) = sum_{k!=j} (w_k/w_j)(f_k - f_j)/(x_j - x_k) (Schneider &
// Werner 1986), and dL/dx_j|w gets -g_p r'(x_j) (r depends on the nodes only
// through x - x_k).  The total node gradient adds the chain through the
// weights, dL/dx_l += sum_k dL/dw_k dw_k/dx_l.
//
// Passes (all on the caller's stream, no atomics, fixed reduction order):
//   1. per point (lanes own points, nodes streamed as in the evaluation
//      kernel): N, D, E, F -> dL/dx_p and a pass-2 record {x, c, c r,
//      g at a hit, g r' at a hit}; non-finite points get a record far from
//      every node with zero weights (they contribute nothing) and NaN dx_p;
//   2. per node and chunk of points (lanes own nodes, points streamed as
//      wave-uniform scalar loads): S1..S4 and the hit sums, with
//      reciprocals taken four points at a time (simultaneous inversion); a
//      group whose product is not normal (a hit, or extreme range) is redone
//      pair by pair, where a zero difference adds the hit terms;
//   3. per node and field: fixed-order sum of the chunk partials; then per
//      node dL/df, dL/dw and the direct dL/dx_k;
//   4. per node: the weight chain (O(d^3) per node), total dL/dx_k.
#include <mutex>
#include <utility>
#include <vector>

#include "bwd_math.h"
#include "fh_internal.h"
#include "pair_math.h"
#include "split_math.h"

namespace fhk {

// ---------------------------------------------------------------- pass 1 --
// DERIV: the derivative r'(x) = (r E - F) / D of the interpolant (dL/dx_p
// with g_p = 1; the node formula at hits) is written to dx and r to r_out;
// g, the records and the padding are not used (m_pad = m).  EF: E and F are
// summed (for dx; without them pass 1 writes only the records).  SAVE (with
// neither): the forward of the saved-state adjoint -- r to r_out and the
// records for g_p = 1 with r in place of c r: {x, 1/D, r, 1 at a hit,
// r'(x_j) at a hit}, which k_bwd_scale_records later scales by g.
template <int P, bool DERIV, bool EF, bool SAVE = false>
__global__ void __launch_bounds__(256)
    k_bwd_points(const double* __restrict__ x, const double* __restrict__ g, int64_t m,
                 int64_t m_pad, const double* __restrict__ tx, const double* __restrict__ tw,
                 const double* __restrict__ twf, const double* __restrict__ tf, int64_t n_pad,
                 int64_t n, double* __restrict__ dx, PointRecs rec, double* __restrict__ r_out) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * P + threadIdx.x;
  // a point far outside the node range: its differences are all of the
  // order of the span, never zero
  const double span = tx[n - 1] - tx[0];
  const double far = tx[n - 1] + span + 1.0;
  double xp[P], N[P], D[P], E[P], F[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + (int64_t)j * blockDim.x;
    xp[j] = idx < m ? x[idx] : far;
    N[j] = D[j] = E[j] = F[j] = 0.0;
  }
  // 32-bit counter keeps loop control on the scalar unit; no range test in
  // the loop: a zero, infinite or NaN group product makes every t of its
  // group NaN, and with it D (tested once per point below)
  for (int k = 0; k < (int)n_pad; k += 8) {
    double xk[8], wk[8], vk[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      xk[i] = tx[k + i];
      wk[i] = tw[k + i];
      vk[i] = twf[k + i];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      double dl[8], t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) dl[i] = xp[j] - xk[i];
      group_product_reciprocals<8>(dl, t);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        D[j] = __builtin_fma(wk[i], t[i], D[j]);
        N[j] = __builtin_fma(vk[i], t[i], N[j]);
        if constexpr (EF) {
          const double t2 = t[i] * t[i];
          E[j] = __builtin_fma(wk[i], t2, E[j]);
          F[j] = __builtin_fma(vk[i], t2, F[j]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t idx = base + (int64_t)j * blockDim.x;
    if (idx >= m_pad) continue;
    const bool bad = !(fabs(D[j]) <= 0x1.fffffffffffffp+1023);
    if (idx >= m) {
      if (!DERIV) {
        rec.x[idx] = far; rec.c[idx] = 0.0; rec.cr[idx] = 0.0; rec.hg[idx] = 0.0;
        rec.hgr[idx] = 0.0;
      }
      continue;
    }
    const double gp = (DERIV || SAVE) ? 1.0 : g[idx];
    const double t = xp[j];
    double dxp, rv, c = 0.0, cr = 0.0, hg = 0.0, hgr = 0.0, xr = t;
    if (!__builtin_isfinite(t)) {
      dxp = rv = __builtin_nan("");
      xr = far;
    } else if (!bad) {
      rv = N[j] / D[j];
      c = gp / D[j];
      cr = c * rv;
      dxp = EF ? c * (rv * E[j] - F[j]) : 0.0;
    } else {
      // pair-by-pair: exact hit or extreme range
      bwd_point_exact(t, gp, tx, tw, tf, n, &dxp, &c, &cr, &hg, &hgr, &rv);
    }
    if (EF && dx) dx[idx] = dxp;
    if (DERIV) {
      if (r_out) r_out[idx] = rv;
    } else if (SAVE) {
      r_out[idx] = rv;
      rec.x[idx] = xr; rec.c[idx] = c; rec.cr[idx] = rv; rec.hg[idx] = hg; rec.hgr[idx] = hgr;
    } else {
      rec.x[idx] = xr; rec.c[idx] = c; rec.cr[idx] = cr; rec.hg[idx] = hg; rec.hgr[idx] = hgr;
    }
  }
}

// ---------------------------------------------------------------- pass 2 --
// grid: x = node tile groups, y = groups of four chunks of `chunk` points
// (chunk a multiple of G); wave w of the block takes chunk 4*blockIdx.y + w
// and the node tiles (64*Q nodes each) blockIdx.x, blockIdx.x + gridDim.x,
// ...  Reciprocals are taken G points at a time.  SUMS: 2 all four node
// sums and both hit sums (the node gradient needs them), 1 S1 and H1 only
// (dL/df; the others written as zeros), 0 none (no node partials written).
// PT (G = 8, saved-state adjoint): also the point side of the same pairs,
// sum_k (w_k r_p - w_k f_k) t_pk^2 = dL/dx_p / c_p (rr = r_p), summed over
// the wave's nodes across lanes (wave_sum8, through LDS) and over its tiles
// in place: gpart[blockIdx.x][p] (each wave owns its chunk's slots of its
// tile group; the lane that adds a slot is the lane that wrote it).  Padding nodes
// (k >= n) sit far beyond the last node with zero weight: they add nothing,
// and never make a group product zero.
template <int Q, int G, int SUMS, bool PT>
__global__ void __launch_bounds__(256)
    k_bwd_nodes(const double* __restrict__ rec_x, const double* __restrict__ rec_c,
                const double* __restrict__ rec_cr, const double* __restrict__ rec_hg,
                const double* __restrict__ rec_hgr, const double* __restrict__ rr, int64_t chunk,
                int64_t chunks, const double* __restrict__ tx, const double* __restrict__ tw,
                const double* __restrict__ twf, int64_t n, int64_t n_pad,
                double* __restrict__ part, double* __restrict__ gpart, int64_t m_pad) {
  static_assert(!PT || G == 8, "the point-side sums run over groups of eight points");
  __shared__ double red[PT ? 4 : 1][PT ? 8 * 64 : 1];
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c >= chunks) return;
  const int64_t tiles = (n_pad + 64 * Q - 1) / (64 * Q);
  const int64_t p0 = c * chunk;
  // the records are read-only here: wave-uniform scalar loads
  const double* rx = rec_x + p0;
  const double* rc = rec_c + p0;
  const double* rcr = rec_cr + p0;
  // beyond the far point of pass 1's padding records as well
  const double far = tx[n - 1] + 2.0 * ((tx[n - 1] - tx[0]) + 1.0);
  const int slot = lane >> 3;
  double* lds = red[PT ? threadIdx.x >> 6 : 0];
  double* __restrict__ gp_out = PT ? gpart + (int64_t)blockIdx.x * m_pad + p0 : nullptr;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const bool first = tile == (int64_t)blockIdx.x;
    const int64_t k0 = tile * 64 * Q + lane;
    double xk[Q], wk[Q], wfk[Q], S1[Q], S2[Q], S3[Q], S4[Q], H1[Q], H2[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t k = k0 + q * 64;
      const bool real = k < n;
      xk[q] = real ? tx[k] : far;
      wk[q] = PT && real ? tw[k] : 0.0;
      wfk[q] = PT && real ? twf[k] : 0.0;
      S1[q] = S2[q] = S3[q] = S4[q] = H1[q] = H2[q] = 0.0;
    }
    for (int p = 0; p < (int)chunk; p += G) {
      double px[G], pc[G], pcr[G], pr[G], gs[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        px[i] = rx[p + i];
        pc[i] = SUMS >= 1 ? rc[p + i] : 0.0;
        pcr[i] = SUMS == 2 ? rcr[p + i] : 0.0;
        pr[i] = PT ? rr[p0 + p + i] : 0.0;
        gs[i] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double dl[G], t[G];
#pragma unroll
        for (int i = 0; i < G; ++i) dl[i] = px[i] - xk[q];
        const bool bad = group_reciprocals<G>(dl, t);
        if (!bad) {
#pragma unroll
          for (int i = 0; i < G; ++i) {
            if constexpr (SUMS >= 1) S1[q] = __builtin_fma(pc[i], t[i], S1[q]);
            if constexpr (SUMS == 2 || PT) {
              const double t2 = t[i] * t[i];
              if constexpr (SUMS == 2) {
                S2[q] = __builtin_fma(pcr[i], t[i], S2[q]);
                S3[q] = __builtin_fma(pc[i], t2, S3[q]);
                S4[q] = __builtin_fma(pcr[i], t2, S4[q]);
              }
              if constexpr (PT)
                gs[i] = __builtin_fma(__builtin_fma(wk[q], pr[i], -wfk[q]), t2, gs[i]);
            }
          }
        } else {
          // pair by pair: a zero difference is a hit on this node
          for (int i = 0; i < G; ++i)
            bwd_pair_exact<SUMS, PT>(px[i], pc[i], pcr[i], rec_hg[p0 + p + i],
                                     rec_hgr[p0 + p + i], xk[q], S1[q], S2[q], S3[q], S4[q],
                                     H1[q], H2[q], wk[q], wfk[q], pr[i], &gs[i]);
        }
      }
      if constexpr (PT) {
        const double z = wave_sum8(gs, lds);
        if ((lane & 7) == 0) {
          double* o = gp_out + p + slot;
          *o = first ? z : *o + z;
        }
      }
    }
    if constexpr (SUMS >= 1) {
      double* out = part + c * kPartFields * n_pad;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t k = k0 + q * 64;
        if (k >= n_pad) continue;
        out[0 * n_pad + k] = S1[q];
        out[1 * n_pad + k] = S2[q];
        out[2 * n_pad + k] = S3[q];
        out[3 * n_pad + k] = S4[q];
        out[4 * n_pad + k] = H1[q];
        out[5 * n_pad + k] = H2[q];
      }
    }
  }
}

// Saved-state adjoint, before pass 2: the records for the loss weights g
// from the forward's records for g = 1 (saved: {x, 1/D, r, 1 at a hit,
// r'(x_j) at a hit}; rec.x is saved.x): c = g / D, c r, g and g r'(x_j) at
// a hit, zeros for padding and for points the forward set aside (1/D = 0).
__global__ void __launch_bounds__(256)
    k_bwd_scale_records(PointRecs saved, const double* __restrict__ g, int64_t m, int64_t m_pad,
                        PointRecs rec) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m_pad) return;
  const double gp = p < m ? g[p] : 0.0;
  const double inv_d = saved.c[p];
  const bool hit = saved.hg[p] != 0.0;
  const double c = inv_d == 0.0 ? 0.0 : gp * inv_d;
  rec.c[p] = c;
  rec.cr[p] = inv_d == 0.0 ? 0.0 : c * saved.cr[p];
  rec.hg[p] = hit ? gp : 0.0;
  rec.hgr[p] = hit ? gp * saved.hgr[p] : 0.0;
}

// Saved-state adjoint whose forward kept r'(x_p): dL/dx_p = g_p r'(x_p) (NaN
// at a NaN or infinite point, whose r' is NaN; the node formula at a hit).
__global__ void __launch_bounds__(256)
    k_bwd_point_grad_from_derivative(const double* __restrict__ g,
                                     const double* __restrict__ dr, int64_t m,
                                     double* __restrict__ dx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m) dx[p] = g[p] * dr[p];
}

// Saved-state adjoint, after pass 2: dL/dx_p = c_p times the point-side sum
// over the tile groups (fixed order); g_p r'(x_j) at a hit, NaN at a NaN or
// infinite point.
__global__ void __launch_bounds__(256)
    k_bwd_point_grad(const double* __restrict__ x, const double* __restrict__ g, int64_t m,
                     int64_t m_pad, PointRecs saved, const double* __restrict__ c,
                     const double* __restrict__ gpart, int32_t groups, double* __restrict__ dx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const double xp = x[p];
  double v;
  if (!__builtin_isfinite(xp)) {
    v = __builtin_nan("");
  } else if (saved.hg[p] != 0.0) {
    v = g[p] * saved.hgr[p];
  } else {
    double acc = 0.0;
    for (int32_t j = 0; j < groups; ++j) acc += gpart[(int64_t)j * m_pad + p];
    v = c[p] * acc;
  }
  dx[p] = v;
}

// ---------------------------------------------------------------- pass 3 --
// Sum of the chunk partials of one field for 64 nodes: grid (node tiles of
// 64, kPartFields), wave w of the block adds chunks w, w + 4, ...; the four
// wave sums are combined in a fixed order (deterministic).
__global__ void __launch_bounds__(256)
    k_bwd_reduce(const double* __restrict__ part, int64_t chunks, int64_t n_pad,
                 double* __restrict__ sums) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  const int v = blockIdx.y;
  double acc = 0.0;
  if (k < n_pad)
    for (int64_t c = w; c < chunks; c += 4) acc += part[(c * kPartFields + v) * n_pad + k];
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && k < n_pad) sums[v * n_pad + k] = ((red[0][lane] + red[1][lane]) + red[2][lane]) +
                                                 red[3][lane];
}

// The S sums may carry a common factor 2^e (the precision-split passes run
// with c_p scaled by the weight scale 2^e, see backward_split.hip; e = 0
// when scale_exp is null): dL/df = w 2^-e S1 + H1, dL/dw = 2^-e (f S1 - S2),
// dL/dx_k|w = w 2^-e (f S3 - S4) - H2.  Scaling by a power of two is exact.
__global__ void __launch_bounds__(64)
    k_bwd_finish(const double* __restrict__ sums, int64_t n_pad, int64_t n,
                 const double* __restrict__ tw, const double* __restrict__ tf,
                 const int32_t* __restrict__ scale_exp, double* __restrict__ df,
                 double* __restrict__ dw, double* __restrict__ dxd) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = scale_exp ? *scale_exp : 0;
  double s[kPartFields];
#pragma unroll
  for (int v = 0; v < kPartFields; ++v) s[v] = sums[v * n_pad + k];
  const double w = ldexp(tw[k], -e), f = tf[k];
  if (df) df[k] = w * s[0] + s[4];
  dw[k] = ldexp(f * s[0] - s[1], -e);
  dxd[k] = w * (f * s[2] - s[3]) - s[5];
}

// ---------------------------------------------------------------- pass 4 --
// dL/dx_l = direct term + sum over the weights that depend on x_l:
// w_k = sum_{i in J_k} T_{k,i},  T_{k,i} = (-1)^i / prod_{j in [i,i+d], j!=k} (x_k - x_j),
// dT/dx_l = T / (x_k - x_l) for l != k in the window, dT/dx_k = -T sum_{j!=k} 1/(x_k - x_j).
// One wave per node l; its lanes take the (k, i) pairs with x_l in window i
// (k within d of l), each O(d); the wave sum runs in a fixed butterfly order.
__global__ void __launch_bounds__(256)
    k_bwd_chain(const double* __restrict__ x, int64_t n, int32_t d, const double* __restrict__ dw,
                const double* __restrict__ dxd, double* __restrict__ dxn) {
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (l >= n) return;  // whole wave
  const int64_t klo = l - d > 0 ? l - d : 0;
  const int64_t khi = l + d < n - 1 ? l + d : n - 1;
  const int64_t combos = (khi - klo + 1) * (int64_t)(d + 1);
  double acc = 0.0;
  for (int64_t q = lane; q < combos; q += 64) {
    const int64_t k = klo + q / (d + 1);
    const int64_t i = k - d + q % (d + 1);  // window start, i in [k-d, k]
    if (i < 0 || i > n - 1 - d || l < i || l > i + d) continue;
    double prod = 1.0;
    for (int64_t j = i; j <= i + d; ++j)
      if (j != k) prod *= (x[k] - x[j]);
    double T = 1.0 / prod;
    if (i & 1) T = -T;
    double dT;
    if (l != k) {
      dT = T / (x[k] - x[l]);
    } else {
      double inv = 0.0;
      for (int64_t j = i; j <= i + d; ++j)
        if (j != k) inv += 1.0 / (x[k] - x[j]);
      dT = -T * inv;
    }
    acc = __builtin_fma(dw[k], dT, acc);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) dxn[l] = dxd[l] + acc;
}

// ------------------------------------------------------------- launcher --
// Blocks of 256 threads of `kernel` resident on the current device at once
// (over all CUs); 2048 when the runtime cannot tell (no device).
static int64_t resident_blocks(const void* kernel) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<int, const void*>, int64_t>> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2048;
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& e : cache)
    if (e.first.first == dev && e.first.second == kernel) return e.second;
  int cus = 0, per_cu = 0;
  int64_t r = 2048;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) == hipSuccess &&
      cus > 0 && per_cu > 0)
    r = (int64_t)cus * per_cu;
  cache.push_back({{dev, kernel}, r});
  return r;
}

// The five record arrays of a PointRecs as kernel arguments.
#define FH_RECS(r) (r).x, (r).c, (r).cr, (r).hg, (r).hgr

static const void* bwd_nodes_kernel(int q, int g, bool saved) {
  if (saved) return reinterpret_cast<const void*>(k_bwd_nodes<2, 8, 2, true>);
  switch (q * 10 + g) {
    case 14: return reinterpret_cast<const void*>(k_bwd_nodes<1, 4, 2, false>);
    case 24: return reinterpret_cast<const void*>(k_bwd_nodes<2, 4, 2, false>);
    case 18: return reinterpret_cast<const void*>(k_bwd_nodes<1, 8, 2, false>);
    default: return reinterpret_cast<const void*>(k_bwd_nodes<2, 8, 2, false>);
  }
}

BackwardPlan plan_backward(int64_t n, int64_t m, bool split, bool saved) {
  BackwardPlan p;
  p.n_pad = round_up(n, kNodePad);
  p.split = split;
  saved = saved && !split;
  // binary64: two points per lane in pass 1, two nodes per lane and
  // inversion over eight points in pass 2 (measured best on the 2049-node
  // gradient workload); split: one node per lane up to 4096 nodes
  p.p = 2;
  p.g = 8;
  p.q = split ? (p.n_pad >= 4096 ? 2 : 1) : 2;
  // Pass 2 runs (node tile, chunk) units of equal work.  The chunk count is
  // chosen so that all units are resident at once (one full round): a
  // second, partly filled round would leave most of the chip idle for as
  // long as the first.  binary64: blocks of four waves, each a 64 q node
  // tile and one chunk; split: blocks of 256 q nodes sharing one chunk.
  p.groups = 0;
  int64_t chunks;
  if (split) {
    const int64_t tiles = (p.n_pad + 256 * p.q - 1) / (256 * p.q);
    const int64_t rows = resident_blocks(bwd_nodes_split_kernel(p.q)) / tiles;
    chunks = rows > 1 ? rows : 1;
  } else {
    // saved-state adjoint: a wave takes every groups-th tile for its chunk
    const int64_t tiles = (p.n_pad + 64 * p.q - 1) / (64 * p.q);
    p.groups = saved ? (int32_t)(tiles < kMaxTileGroups ? tiles : kMaxTileGroups) : 0;
    const int64_t rows =
        resident_blocks(bwd_nodes_kernel(p.q, p.g, saved)) / (saved ? p.groups : tiles);
    chunks = 4 * (rows > 1 ? rows : 1);
  }
  const int64_t align = split ? kTile : 8;
  const int64_t max_chunks = (m + 255) / 256;  // chunks of >= 256 points
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  p.chunk = round_up((m + chunks - 1) / chunks, align);
  if (p.chunk < align) p.chunk = align;
  p.chunks = (m + p.chunk - 1) / p.chunk;
  if (p.chunks < 1) p.chunks = 1;
  p.m_pad = p.chunks * p.chunk;
  return p;
}

size_t layout_backward(void* ws, int64_t n, int64_t m, bool split, NodeTable* t,
                       BackwardBufs* b, bool saved) {
  size_t off = layout_tables(ws, n, t);
  const BackwardPlan p = plan_backward(n, m, split, saved);
  char* base = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return q;
  };
  b->plan = p;
  double** fields[] = {&b->rec.x, &b->rec.c, &b->rec.cr, &b->rec.hg, &b->rec.hgr};
  for (double** f : fields) *f = reinterpret_cast<double*>(take(sizeof(double) * p.m_pad));
  b->rec32 = split ? reinterpret_cast<float4*>(take(sizeof(float4) * p.m_pad)) : nullptr;
  b->part = reinterpret_cast<double*>(take(sizeof(double) * kPartFields * p.n_pad * p.chunks));
  b->sums = reinterpret_cast<double*>(take(sizeof(double) * kPartFields * p.n_pad));
  b->dw = reinterpret_cast<double*>(take(sizeof(double) * p.n_pad));
  b->dxd = reinterpret_cast<double*>(take(sizeof(double) * p.n_pad));
  b->saved = PointRecs{};
  b->gpart = nullptr;
  b->saved32 = nullptr;
  if (saved) {
    // the forward's records (g = 1) share the point coordinates with rec
    b->saved.x = b->rec.x;
    double** sf[] = {&b->saved.c, &b->saved.cr, &b->saved.hg, &b->saved.hgr};
    for (double** f : sf) *f = reinterpret_cast<double*>(take(sizeof(double) * p.m_pad));
    if (p.groups > 0)
      b->gpart = reinterpret_cast<double*>(take(sizeof(double) * p.groups * p.m_pad));
    if (split) b->saved32 = reinterpret_cast<float4*>(take(sizeof(float4) * p.m_pad));
  }
  return off;
}

template <int P>
static void launch_bwd_points_p(const BackwardPlan& p, const double* x, const double* g,
                                int64_t m, const NodeTable& t, int64_t n, double* dx,
                                const PointRecs& rec, hipStream_t s) {
  const dim3 grid((unsigned)((p.m_pad + 256 * P - 1) / (256 * P)));
  if (dx)
    k_bwd_points<P, false, true><<<grid, 256, 0, s>>>(x, g, m, p.m_pad, t.x, t.w, t.wf, t.f,
                                                      t.n_pad, n, dx, rec, nullptr);
  else
    k_bwd_points<P, false, false><<<grid, 256, 0, s>>>(x, g, m, p.m_pad, t.x, t.w, t.wf, t.f,
                                                       t.n_pad, n, dx, rec, nullptr);
}

// dx null: E and F are not summed (the records are all pass 2 needs)
static hipError_t launch_bwd_points(const BackwardPlan& p, const double* x, const double* g,
                                    int64_t m, const NodeTable& t, int64_t n, double* dx,
                                    const PointRecs& rec, hipStream_t s) {
  switch (p.p) {
    case 1: launch_bwd_points_p<1>(p, x, g, m, t, n, dx, rec, s); break;
    case 2: launch_bwd_points_p<2>(p, x, g, m, t, n, dx, rec, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// full: all four sums (the node gradient is wanted), else S1 only
static hipError_t launch_bwd_nodes(const BackwardPlan& p, const PointRecs& rec, const NodeTable& t,
                                   int64_t n, double* part, bool full, hipStream_t s) {
  const dim3 grid((unsigned)((p.n_pad + 64 * p.q - 1) / (64 * p.q)),
                  (unsigned)((p.chunks + 3) / 4));
  const int v = p.q * 10 + p.g;
  switch (v) {
#define FH_NODES_CASE(Q, G)                                                                 \
  case Q * 10 + G:                                                                        \
    if (full)                                                                             \
      k_bwd_nodes<Q, G, 2, false><<<grid, 256, 0, s>>>(FH_RECS(rec), nullptr, p.chunk,    \
                                                       p.chunks, t.x, t.w, t.wf, n, t.n_pad, \
                                                       part, nullptr, p.m_pad);           \
    else                                                                                  \
      k_bwd_nodes<Q, G, 1, false><<<grid, 256, 0, s>>>(FH_RECS(rec), nullptr, p.chunk,    \
                                                       p.chunks, t.x, t.w, t.wf, n, t.n_pad, \
                                                       part, nullptr, p.m_pad);           \
    break;
    FH_NODES_CASE(1, 4)
    FH_NODES_CASE(2, 4)
    FH_NODES_CASE(1, 8)
    FH_NODES_CASE(2, 8)
#undef FH_NODES_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_node_tail(const double* nodes, int64_t n, int32_t d, const NodeTable& t,
                                   const BackwardBufs& b, const int32_t* scale_exp, double* df,
                                   double* dxn, hipStream_t s);

hipError_t launch_backward(const double* nodes, const double* x, const double* g, int64_t n,
                           int32_t d, int64_t m, const NodeTable& t, const BackwardBufs& b,
                           const int32_t* scale_exp, double* df, double* dx, double* dxn,
                           hipStream_t s) {
  const BackwardPlan& p = b.plan;
  hipError_t e;
  // only the passes and sums the requested gradients need: dL/dx_p comes
  // from pass 1 alone; dL/df needs S1 (and the hit sums); the node gradient
  // all four sums
  const bool nodes_pass = df != nullptr || dxn != nullptr, full = dxn != nullptr;
  if (p.split) {
    e = launch_backward_split_passes(x, g, n, m, t, b, scale_exp, dx, nodes_pass, full, s);
    if (e != hipSuccess) return e;
  } else {
    e = launch_bwd_points(p, x, g, m, t, n, dx, b.rec, s);
    if (e != hipSuccess) return e;
    if (nodes_pass) {
      e = launch_bwd_nodes(p, b.rec, t, n, b.part, full, s);
      if (e != hipSuccess) return e;
    }
  }
  if (!nodes_pass) return hipSuccess;
  return launch_node_tail(nodes, n, d, t, b, p.split ? scale_exp : nullptr, df, dxn, s);
}

// Passes 3 and 4 from the chunk partials of pass 2.
static hipError_t launch_node_tail(const double* nodes, int64_t n, int32_t d, const NodeTable& t,
                                   const BackwardBufs& b, const int32_t* scale_exp, double* df,
                                   double* dxn, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  hipError_t e;
  const dim3 g3((unsigned)((p.n_pad + 63) / 64), (unsigned)kPartFields);
  k_bwd_reduce<<<g3, 256, 0, s>>>(b.part, p.chunks, p.n_pad, b.sums);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // per-node passes in 64-thread blocks: n is small, so spread it over CUs
  const dim3 g4((unsigned)((n + 63) / 64));
  k_bwd_finish<<<g4, 64, 0, s>>>(b.sums, p.n_pad, n, t.w, t.f, scale_exp, df, b.dw, b.dxd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dxn) {
    k_bwd_chain<<<dim3((unsigned)((n + 3) / 4)), 256, 0, s>>>(nodes, n, d, b.dw, b.dxd, dxn);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_backward_tail(const double* nodes, int64_t n, int32_t d, const NodeTable& t,
                                const BackwardBufs& b, const int32_t* scale_exp, double* df,
                                double* dxn, hipStream_t s) {
  return launch_node_tail(nodes, n, d, t, b, scale_exp, df, dxn, s);
}

// --------------------------------------------------- saved-state adjoint --
hipError_t launch_forward_saved(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                const BackwardBufs& b, double* r, double* dr, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  if (p.groups <= 0) return hipErrorInvalidValue;
  constexpr int P = 2;
  const dim3 grid((unsigned)((p.m_pad + 256 * P - 1) / (256 * P)));
  if (dr)  // E and F as well: r' = (r E - F) / D, the derivative pass's bits
    k_bwd_points<P, false, true, true><<<grid, 256, 0, s>>>(
        x, nullptr, m, p.m_pad, t.x, t.w, t.wf, t.f, t.n_pad, n, dr, b.saved, r);
  else
    k_bwd_points<P, false, false, true><<<grid, 256, 0, s>>>(
        x, nullptr, m, p.m_pad, t.x, t.w, t.wf, t.f, t.n_pad, n, nullptr, b.saved, r);
  return hipGetLastError();
}

hipError_t launch_point_grad_from_derivative(const double* g, const double* dr, int64_t m,
                                             double* dx, hipStream_t s) {
  if (m == 0) return hipSuccess;
  k_bwd_point_grad_from_derivative<<<dim3((unsigned)((m + 255) / 256)), 256, 0, s>>>(g, dr, m,
                                                                                  dx);
  return hipGetLastError();
}

hipError_t launch_backward_saved(const double* nodes, const double* x, const double* dr,
                                 const double* g, int64_t n, int32_t d, int64_t m,
                                 const NodeTable& t, const BackwardBufs& b, double* df,
                                 double* dx, double* dxn, hipStream_t s) {
  const BackwardPlan& p = b.plan;
  if (p.groups <= 0) return hipErrorInvalidValue;
  if (m == 0) dx = nullptr;  // no points: node sums of the padding records (zeros) only
  hipError_t e;
  if (dx && dr) {  // the forward kept r': no point-side sums in the pass below
    if ((e = launch_point_grad_from_derivative(g, dr, m, dx, s)) != hipSuccess) return e;
    dx = nullptr;
  }
  if (df == nullptr && dx == nullptr && dxn == nullptr) return hipSuccess;
  k_bwd_scale_records<<<dim3((unsigned)((p.m_pad + 255) / 256)), 256, 0, s>>>(b.saved, g, m,
                                                                              p.m_pad, b.rec);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int sums = dxn ? 2 : (df ? 1 : 0);
  const bool pt = dx != nullptr;
  const dim3 grid((unsigned)p.groups, (unsigned)((p.chunks + 3) / 4));
#define FH_SAVED_CASE(S, PT)                                                                 \
  if (sums == S && pt == PT)                                                                \
    k_bwd_nodes<2, 8, S, PT><<<grid, 256, 0, s>>>(FH_RECS(b.rec), b.saved.cr, p.chunk,      \
                                                  p.chunks, t.x, t.w, t.wf, n, t.n_pad,     \
                                                  b.part, b.gpart, p.m_pad);
  FH_SAVED_CASE(2, true)
  FH_SAVED_CASE(2, false)
  FH_SAVED_CASE(1, true)
  FH_SAVED_CASE(1, false)
  FH_SAVED_CASE(0, true)
#undef FH_SAVED_CASE
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dx) {
    k_bwd_point_grad<<<dim3((unsigned)((m + 255) / 256)), 256, 0, s>>>(
        x, g, m, p.m_pad, b.saved, b.rec.c, b.gpart, p.groups, dx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (sums == 0) return hipSuccess;
  return launch_node_tail(nodes, n, d, t, b, nullptr, df, dxn, s);
}

// ---------------------------------------------------------- derivative --
hipError_t launch_eval_deriv(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                             double* dr, hipStream_t s) {
  if (m == 0) return hipSuccess;
  constexpr int P = 2;
  const dim3 grid((unsigned)((m + 256 * P - 1) / (256 * P)));
  k_bwd_points<P, true, true><<<grid, 256, 0, s>>>(x, nullptr, m, m, t.x, t.w, t.wf, t.f,
                                                   t.n_pad, n, dr, PointRecs{}, r);
  return hipGetLastError();
}

}  // namespace fhk
