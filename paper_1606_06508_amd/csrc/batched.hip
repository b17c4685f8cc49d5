// Batched evaluation: many interpolants of uneven n and d in one captured
// HIP graph (gfx950).
//
// Layout.  The caller's arrays are CSR: instance i owns nodes/values
// [noff_i, noff_i + n_i) and points/outputs [poff_i, poff_i + m_i).  The
// batch builds one concatenated node table (x, w, w f, f in binary64 and the
// binary32 split records), each instance padded to a multiple of 8 records
// with zero-weight copies of its last node.
//
// Work.  A work item is one strip of 256 * P consecutive points of one
// instance (one block's worth).  Items are ordered longest first (by the
// instance's padded node count, i.e. the cost of a strip), and a persistent
// grid sized to the resident capacity of the device pulls them from an
// atomic counter: big strips start first, small ones fill the tail.  Inside
// an item the block runs the same node loops as the single-interpolant
// kernels (binary64: each wave streams the instance's node records through
// scalar loads; split: the block stages them in LDS).  The batch's weights
// are the library's, which alternate in sign, so the split kernel takes its
// sums by node tiles (one binary32 multiply-add per pair into the tile's
// even or odd sum serves D and the Lebesgue sum; the tile around each point
// is corrected afterwards), with or without Lambda, so r does not depend on
// it.  The binary64 kernel keeps plain sums: by blocks of 16 its r-only
// form ran 4 % slower on the 4096-instance workload, with Lambda 2.5 %
// faster.
//
// Graph.  fh_batch_create captures, on a private stream: a one-thread kernel
// that resets the item counter (a kernel rather than a memset node), the
// weight/packing pass for all instances, the split packing pass if needed,
// and the persistent evaluation kernel.  fh_eval_batched is one
// hipGraphLaunch.
#include <algorithm>
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
  int32_t shift, pad;  // split: ef - e of the instance's table (written by its packing)
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
// binary32 records (see k_pack_split for the scaling argument)
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

template <int P, bool R, bool L>
__global__ void __launch_bounds__(256)
    k_batch_f64(const InstDesc* __restrict__ inst, const int2* __restrict__ items, int n_items,
                uint32_t* counter, const double* __restrict__ x, double* __restrict__ r,
                double* __restrict__ lam, const double* __restrict__ tx,
                const double* __restrict__ tw, const double* __restrict__ twf,
                const double* __restrict__ tf) {
  constexpr int G = 8;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (;;) {
    const int item = next_item(counter, &s_item);
    if (item >= n_items) break;
    const int2 it = items[item];
    const InstDesc ds = inst[__builtin_amdgcn_readfirstlane(it.x)];
    const int64_t strip = __builtin_amdgcn_readfirstlane(it.y);
    const double* px = x + ds.poff;
    const int64_t base = strip * 256 * P + tid;
    double xp[P], N[P], D[P], A[P];
    bool bad[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t idx = base + j * 256;
      xp[j] = px[idx < ds.m ? idx : ds.m - 1];
      N[j] = D[j] = A[j] = 0.0;
      bad[j] = false;
    }
    accumulate_f64<P, G, R, L>(xp, tx + ds.toff, tw + ds.toff, twf + ds.toff, 0, ds.n_pad, N, D,
                               A, bad);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t idx = base + j * 256;
      if (idx >= ds.m) continue;
      double rv, lv;
      if (bad[j]) {
        const PointRL e =
            eval_point_exact<R, L>(xp[j], tx + ds.toff, tw + ds.toff, tf + ds.toff, ds.n);
        rv = e.r;
        lv = e.l;
      } else {
        rv = ldexp(N[j] / D[j], ds.shift);
        lv = A[j] / fabs(D[j]);
      }
      if (R) r[ds.poff + idx] = rv;
      if (L) lam[ds.poff + idx] = lv;
    }
  }
}

template <int P, bool R, bool L>
__global__ void __launch_bounds__(kStage)
    k_batch_split(const InstDesc* __restrict__ inst, const int2* __restrict__ items, int n_items,
                  uint32_t* counter, const double* __restrict__ x, double* __restrict__ r,
                  double* __restrict__ lam, const float4* __restrict__ s4,
                  const double* __restrict__ tx, const double* __restrict__ tw,
                  const double* __restrict__ tf) {
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
    const int64_t base = strip * kStage * P + tid;
    const double x_first = tx[ds.toff], x_last = tx[ds.toff + ds.n - 1];
    double xp[P], N[P], D[P], A[P];
    float xh[P], xl[P];
    bool bad[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t idx = base + j * kStage;
      xp[j] = px[idx < ds.m ? idx : ds.m - 1];
      xh[j] = (float)xp[j];
      xl[j] = (float)(xp[j] - (double)xh[j]);
      N[j] = D[j] = A[j] = 0.0;
      bad[j] = !in_split_domain(xp[j], x_first, x_last);
    }
    split_block_sums<P, R, L, 4, true>(stage, s4 + ds.toff, ds.n_pad, mask, xh, xl, N, D, A, bad);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t idx = base + j * kStage;
      if (idx >= ds.m) continue;
      double rv, lv;
      if (bad[j]) {
        const PointRL e =
            eval_point_exact<R, L>(xp[j], tx + ds.toff, tw + ds.toff, tf + ds.toff, ds.n);
        rv = e.r;
        lv = e.l;
      } else {
        double a = A[j];
        if constexpr (L)
          a = split_tile_fix<4>(xp[j], xh[j], xl[j], tx + ds.toff, ds.n, s4 + ds.toff, ds.n_pad,
                                mask, a);
        rv = ldexp(N[j] / D[j], ds.shift);
        lv = a / fabs(D[j]);
      }
      if (R) r[ds.poff + idx] = rv;
      if (L) lam[ds.poff + idx] = lv;
    }
    __syncthreads();  // the next item's staging reuses the LDS buffers
  }
}

int batched_variant_count() { return 3; }
void batched_variant_shape(int id, int* p, int* g, int* s, bool split) {
  static const int P[3] = {1, 2, 4};
  *p = (id >= 0 && id < 3) ? P[id] : 0;
  *g = split ? 4 : 8;  // split: binary32 simultaneous inversion of node quads
  *s = 1;
}

}  // namespace fhk

using namespace fhk;

struct fh_batch {
  int32_t count = 0, prec = 0, variant = 0, points_per_lane = 1;
  int device = 0;
  int64_t total_pad = 0, n_items = 0;
  void* mem = nullptr;
  InstDesc* inst = nullptr;
  int64_t* toff = nullptr;
  int2* items = nullptr;
  uint32_t* ctrl = nullptr;  // [0] item counter, [1] sticky status bits
  double *tx = nullptr, *tw = nullptr, *twf = nullptr, *tf = nullptr;
  float4* s4 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

template <int P>
hipError_t enqueue_eval(fh_batch* b, const double* x, double* r, double* lam, int grid,
                        hipStream_t s) {
  const int n_items = (int)b->n_items;
  if (b->prec == FH_FP32_SPLIT) {
    if (r && lam)
      k_batch_split<P, true, true><<<grid, kStage, 0, s>>>(b->inst, b->items, n_items, b->ctrl, x,
                                                           r, lam, b->s4, b->tx, b->tw, b->tf);
    else if (r)
      k_batch_split<P, true, false><<<grid, kStage, 0, s>>>(b->inst, b->items, n_items, b->ctrl,
                                                            x, r, lam, b->s4, b->tx, b->tw, b->tf);
    else
      k_batch_split<P, false, true><<<grid, kStage, 0, s>>>(b->inst, b->items, n_items, b->ctrl,
                                                            x, r, lam, b->s4, b->tx, b->tw, b->tf);
  } else {
    if (r && lam)
      k_batch_f64<P, true, true><<<grid, 256, 0, s>>>(b->inst, b->items, n_items, b->ctrl, x, r,
                                                      lam, b->tx, b->tw, b->twf, b->tf);
    else if (r)
      k_batch_f64<P, true, false><<<grid, 256, 0, s>>>(b->inst, b->items, n_items, b->ctrl, x, r,
                                                       lam, b->tx, b->tw, b->twf, b->tf);
    else
      k_batch_f64<P, false, true><<<grid, 256, 0, s>>>(b->inst, b->items, n_items, b->ctrl, x, r,
                                                       lam, b->tx, b->tw, b->twf, b->tf);
  }
  return hipGetLastError();
}

template <int P>
int resident_grid(fh_batch* b, bool r, bool l) {
  int per_cu = 0;
  hipError_t e;
  if (b->prec == FH_FP32_SPLIT) {
    const void* k = r && l ? (const void*)k_batch_split<P, true, true>
                           : (r ? (const void*)k_batch_split<P, true, false>
                                : (const void*)k_batch_split<P, false, true>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kStage, 0);
  } else {
    const void* k = r && l ? (const void*)k_batch_f64<P, true, true>
                           : (r ? (const void*)k_batch_f64<P, true, false>
                                : (const void*)k_batch_f64<P, false, true>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0);
  }
  hipDeviceProp_t prop;
  if (e != hipSuccess || hipGetDeviceProperties(&prop, b->device) != hipSuccess) return -1;
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
    b->variant = choose_eval_config(tune_family, avg_n, 0, total_m > 0 ? total_m : 1, true, true)
                     .variant;
    int p, g, s;
    batched_variant_shape(b->variant, &p, &g, &s, prec == FH_FP32_SPLIT);
    b->points_per_lane = p;
  }
  const int64_t strip_pts = 256LL * b->points_per_lane;
  for (int32_t i = 0; i < count; ++i) {
    InstDesc& ds = inst[i];
    ds.noff = noff;
    ds.n = n_host[i];
    ds.d = d_host[i];
    ds.n_pad = round_up(ds.n, kBatchPad);
    ds.toff = total_pad;
    ds.poff = poff;
    ds.m = m_host[i];
    ds.strips = (int32_t)((ds.m + strip_pts - 1) / strip_pts);
    ds.shift = 0;
    ds.pad = 0;
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
  int grid = -1;
  const bool want_r = r_cat != nullptr, want_l = lambda_cat != nullptr;
  switch (b->points_per_lane) {
    case 1: grid = resident_grid<1>(b, want_r, want_l); break;
    case 2: grid = resident_grid<2>(b, want_r, want_l); break;
    default: grid = resident_grid<4>(b, want_r, want_l); break;
  }
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
    if (items > 0) {
      switch (b->points_per_lane) {
        case 1: e = enqueue_eval<1>(b, x_cat, r_cat, lambda_cat, grid, cs); break;
        case 2: e = enqueue_eval<2>(b, x_cat, r_cat, lambda_cat, grid, cs); break;
        default: e = enqueue_eval<4>(b, x_cat, r_cat, lambda_cat, grid, cs); break;
      }
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
