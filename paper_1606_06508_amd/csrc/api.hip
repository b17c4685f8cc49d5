// C ABI of libfh: argument validation, workspace layout, kernel selection and
// launch.  All device work is enqueued on the caller's stream; nothing here
// allocates (the batched entry points, which own device memory, are in
// batched.hip).
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "fh_internal.h"

using namespace fhk;

namespace {

bool sync_check_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("FH_SYNC_CHECK");
    return v && v[0] == '1';
  }();
  return on;
}

fh_status check_problem(const double* nodes, int64_t n, int32_t d) {
  if (n < 1 || n > FH_MAX_NODES || nodes == nullptr) return FH_E_ARG;
  if (d < 0 || (int64_t)d > n - 1) return FH_E_DEGREE;
  return FH_OK;
}

fh_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (ws == nullptr || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return FH_E_WORKSPACE;
  return FH_OK;
}

__global__ void k_clear_word(uint32_t* p) { *p = 0u; }

fh_status status_from_bits(uint32_t bits) {
  if (bits & FH_FLAG_NONFINITE) return FH_E_NONFINITE;
  if (bits & FH_FLAG_NODES) return FH_E_NODES;
  if (bits & FH_FLAG_RANGE) return FH_E_RANGE;
  return FH_OK;
}

fh_status finish(hipError_t e, void* ws, hipStream_t s) {
  if (e != hipSuccess) return FH_E_HIP;
  if (sync_check_enabled()) {
    uint32_t bits = 0;
    return fh_device_status(ws, s, &bits);
  }
  return FH_OK;
}

}  // namespace

namespace {

// The smallest evaluation workspace: the node tables (the octet variants
// also need the room layout_octets reports, else their pair twin runs).
size_t eval_ws_min(int64_t n) {
  fhk::NodeTable t;
  return fhk::layout_tables(nullptr, n, &t);
}

bool octets_usable(int64_t n, int64_t m, size_t ws_bytes) {
  fhk::OctetBufs b;
  return fhk::octets_possible(n, m) && ws_bytes >= fhk::layout_octets(nullptr, n, m, &b);
}

// The tuned variant for the shape; an octet variant gives way to its pair
// twin where its buffers do not fit.
fhk::EvalConfig eval_config(int32_t prec, int64_t n, int64_t m, bool want_r, bool want_l,
                            bool octets) {
  fhk::EvalConfig c = fhk::choose_eval_config(prec, n, 0, m, want_r, want_l);
  if (prec == FH_FP64 && !octets) {
    const int twin = fhk::f64_variant_octet_twin(c.variant);
    if (twin != c.variant && fhk::log_enabled())
      std::fprintf(stderr,
                   "[fh] fp64 n=%lld m=%lld: variant %d has no workspace room for the sorted "
                   "points (fh_workspace_size(FH_OP_EVAL, n, m, ...)): variant %d runs\n",
                   (long long)n, (long long)m, c.variant, twin);
    c.variant = twin;
  }
  return c;
}

}  // namespace

extern "C" {

const char* fh_status_string(int32_t s) {
  switch (s) {
    case FH_OK: return "ok";
    case FH_E_ARG: return "invalid argument";
    case FH_E_DEGREE: return "degree d outside 0..n-1";
    case FH_E_NODES: return "nodes are not strictly increasing";
    case FH_E_NONFINITE: return "a node is not finite";
    case FH_E_RANGE: return "a weight product is not a normal binary64 number";
    case FH_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case FH_E_HIP: return "HIP runtime error";
    case FH_E_UNSUPPORTED: return "combination not supported by the library";
    case FH_E_TOO_LARGE: return "problem exceeds the fixed scratch of fh_eval_noalloc";
    default: return "unknown status";
  }
}

size_t fh_workspace_size(int32_t op, int64_t n, int64_t m, int32_t d, int32_t prec) {
  if (n < 1 || n > FH_MAX_NODES || m < 0 || d < 0 || (int64_t)d > n - 1) return 0;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return 0;
  NodeTable t;
  switch (op) {
    case FH_OP_WEIGHTS: return kStatusBytes;
    case FH_OP_EVAL: {
      // binary64: room for the octet variants' records and m sorted points
      if (prec == FH_FP32_SPLIT) return layout_tables(nullptr, n, &t);
      OctetBufs b;
      return layout_octets(nullptr, n, m, &b);
    }
    case FH_OP_BACKWARD: {
      BackwardBufs b;
      return layout_backward(nullptr, n, m, prec == FH_FP32_SPLIT, &t, &b);
    }
    case FH_OP_BACKWARD_SAVED: {
      BackwardBufs b;
      return layout_backward(nullptr, n, m, prec == FH_FP32_SPLIT, &t, &b, true);
    }
    case FH_OP_LEBESGUE_MAX: {
      LebesgueBufs b;
      return layout_lebesgue_max(nullptr, n, &t, &b);
    }
    default: return 0;
  }
}

fh_status fh_weights(const double* nodes, int64_t n, int32_t d, double* w_out, void* ws,
                     size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (w_out == nullptr) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, kStatusBytes);
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return finish(launch_weights(nodes, n, d, w_out, static_cast<uint32_t*>(ws), s), ws, s);
}

fh_status fh_prepare(const double* nodes, const double* values, int64_t n, int32_t d,
                     const double* w, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, eval_ws_min(n));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  layout_tables(ws, n, &t);
  return finish(launch_pack(nodes, values, w, n, d, t, prec == FH_FP32_SPLIT,
                            static_cast<uint32_t*>(ws), s),
                ws, s);
}

fh_status fh_prepare_many(const double* nodes, const double* values, int64_t n,
                          const int32_t* d_host, int32_t K, int32_t prec, void* const* ws_host,
                          size_t ws_bytes, void* stream) {
  if (n < 1 || n > FH_MAX_NODES || nodes == nullptr || d_host == nullptr || ws_host == nullptr)
    return FH_E_ARG;
  if (K < 1 || K > kPackMany) return FH_E_ARG;
  if (prec == FH_FP32_SPLIT) return FH_E_UNSUPPORTED;
  if (prec != FH_FP64) return FH_E_ARG;
  PackMany a{};
  for (int32_t c = 0; c < K; ++c) {
    const int32_t d = d_host[c];
    if (d < 0 || (int64_t)d > n - 1) return FH_E_DEGREE;
    fh_status st = check_ws(ws_host[c], ws_bytes, eval_ws_min(n));
    if (st != FH_OK) return st;
    for (int32_t e = 0; e < c; ++e)
      if (ws_host[e] == ws_host[c]) return FH_E_ARG;  // one table per workspace
    NodeTable t;
    layout_tables(ws_host[c], n, &t);
    a.x[c] = t.x;
    a.w[c] = t.w;
    a.wf[c] = t.wf;
    a.f[c] = t.f;
    a.pr[c] = t.pr;
    a.pok[c] = t.pok;
    a.status[c] = static_cast<uint32_t*>(ws_host[c]);
    a.d[c] = d;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (launch_pack_many(nodes, values, n, a, K, s) != hipSuccess) return FH_E_HIP;
  if (sync_check_enabled()) {
    for (int32_t c = 0; c < K; ++c) {
      uint32_t bits = 0;
      const fh_status st = fh_device_status(ws_host[c], s, &bits);
      if (st != FH_OK) return st;
    }
  }
  return FH_OK;
}

fh_status fh_eval_prepared_many(void* const* ws_host, size_t ws_bytes, int32_t K, int64_t n,
                                int32_t prec, const double* x, int64_t m, double* const* r_host,
                                double* const* lambda_host, void* stream) {
  if (n < 1 || n > FH_MAX_NODES || m < 0 || (m > 0 && x == nullptr) || ws_host == nullptr)
    return FH_E_ARG;
  if (K < 1 || K > kEvalMany) return FH_E_ARG;
  if (r_host == nullptr && lambda_host == nullptr) return FH_E_ARG;
  if (prec == FH_FP32_SPLIT) return FH_E_UNSUPPORTED;
  if (prec != FH_FP64) return FH_E_ARG;
  EvalMany a{};
  int64_t n_pad = 0;
  for (int32_t c = 0; c < K; ++c) {
    fh_status st = check_ws(ws_host[c], ws_bytes, eval_ws_min(n));
    if (st != FH_OK) return st;
    if ((r_host && r_host[c] == nullptr) || (lambda_host && lambda_host[c] == nullptr))
      return FH_E_ARG;
    NodeTable t;
    layout_tables(ws_host[c], n, &t);
    n_pad = t.n_pad;
    a.x[c] = t.x;
    a.w[c] = t.w;
    a.wf[c] = t.wf;
    a.f[c] = t.f;
    a.pr[c] = t.pr;
    a.pok[c] = t.pok;
    a.alt[c] = static_cast<uint32_t*>(ws_host[c]) + 3;
    a.r[c] = r_host ? r_host[c] : nullptr;
    a.lam[c] = lambda_host ? lambda_host[c] : nullptr;
  }
  if (m == 0) return FH_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the bits of each table are those of one fh_eval_prepared call with m
  // points: the variant tuned for the launch's K * m points is taken only if
  // it sums in the same order as that call's variant
  const bool want_r = r_host != nullptr, want_l = lambda_host != nullptr;
  const bool oct = octets_usable(n, m, ws_bytes);
  const EvalConfig one = eval_config(prec, n, m, want_r, want_l, oct);
  EvalConfig cfg = eval_config(prec, n, m * K, want_r, want_l, oct);
  if (bit_class(prec, cfg.variant) != bit_class(prec, one.variant)) cfg = one;
  const double* xe = x;
  if (f64_variant_octets(cfg.variant)) {
    // every table's octet records, then the points sorted once for all
    OctetTables ot{};
    OctetBufs b0{};
    for (int32_t c = 0; c < K; ++c) {
      OctetBufs b;
      layout_octets(ws_host[c], n, m, &b);
      if (c == 0) b0 = b;
      ot.x[c] = a.x[c];
      ot.w[c] = a.w[c];
      ot.wf[c] = a.wf[c];
      ot.rec[c] = b.rec;
      ot.ok[c] = b.ok;
      a.oc[c] = b.rec;
      a.ook[c] = b.ok;
    }
    a.order = b0.order;
    xe = b0.xs;
    if (launch_octet_records(ot, K, n, n_pad, s) != hipSuccess ||
        launch_sort_points(x, m, a.x[0], n_pad, b0, s) != hipSuccess)
      return FH_E_HIP;
  }
  if (launch_eval_f64_many(xe, m, n, n_pad, a, K, r_host != nullptr, lambda_host != nullptr,
                           cfg, s) != hipSuccess)
    return FH_E_HIP;
  if (sync_check_enabled()) {
    for (int32_t c = 0; c < K; ++c) {
      uint32_t bits = 0;
      const fh_status st = fh_device_status(ws_host[c], s, &bits);
      if (st != FH_OK) return st;
    }
  }
  return FH_OK;
}

fh_status fh_eval_prepared(void* ws, size_t ws_bytes, int64_t n, int32_t prec, const double* x,
                           int64_t m, double* r_out, double* lambda_out, void* stream) {
  if (n < 1 || n > FH_MAX_NODES || m < 0 || (m > 0 && x == nullptr)) return FH_E_ARG;
  if (m > 0 && r_out == nullptr && lambda_out == nullptr) return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  fh_status st = check_ws(ws, ws_bytes, eval_ws_min(n));
  if (st != FH_OK) return st;
  if (m == 0) return FH_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  layout_tables(ws, n, &t);
  const bool oct = prec == FH_FP64 && octets_usable(n, m, ws_bytes);
  const EvalConfig cfg =
      eval_config(prec, n, m, r_out != nullptr, lambda_out != nullptr, oct);
  if (prec == FH_FP32_SPLIT)
    return finish(launch_eval_split(x, m, t, n, static_cast<int32_t*>(ws) + 1,
                                    static_cast<uint32_t*>(ws) + 3, r_out, lambda_out, cfg, s),
                  ws, s);
  OctetArgs oa{};
  const double* xe = x;
  hipError_t e = hipSuccess;
  if (f64_variant_octets(cfg.variant)) {
    OctetBufs b;
    layout_octets(ws, n, m, &b);
    OctetTables ot{};
    ot.x[0] = t.x;
    ot.w[0] = t.w;
    ot.wf[0] = t.wf;
    ot.rec[0] = b.rec;
    ot.ok[0] = b.ok;
    e = launch_octet_records(ot, 1, n, t.n_pad, s);
    if (e == hipSuccess) e = launch_sort_points(x, m, t.x, t.n_pad, b, s);
    oa = OctetArgs{b.rec, b.ok, b.order};
    xe = b.xs;
  }
  if (e == hipSuccess)
    e = launch_eval_f64(xe, m, t, n, static_cast<uint32_t*>(ws) + 3, r_out, lambda_out, cfg, oa,
                        s);
  return finish(e, ws, s);
}

static fh_status eval_common(const double* nodes, const double* values, int64_t n, int32_t d,
                             const double* x, int64_t m, double* r_out, double* lambda_out,
                             const double* w, int32_t prec, void* ws, size_t ws_bytes,
                             void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (m < 0 || (m > 0 && x == nullptr)) return FH_E_ARG;
  if (m > 0 && r_out == nullptr && lambda_out == nullptr) return FH_E_ARG;
  if (r_out != nullptr && values == nullptr) return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, eval_ws_min(n));
  if (st != FH_OK) return st;
  st = fh_prepare(nodes, values, n, d, w, prec, ws, ws_bytes, stream);
  if (st != FH_OK) return st;
  return fh_eval_prepared(ws, ws_bytes, n, prec, x, m, r_out, lambda_out, stream);
}

fh_status fh_eval(const double* nodes, const double* values, int64_t n, int32_t d,
                  const double* x, int64_t m, double* r_out, double* lambda_out, const double* w,
                  int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  if (m > 0 && r_out == nullptr) return FH_E_ARG;
  if (values == nullptr) return FH_E_ARG;
  return eval_common(nodes, values, n, d, x, m, r_out, lambda_out, w, prec, ws, ws_bytes, stream);
}

fh_status fh_lebesgue(const double* nodes, int64_t n, int32_t d, const double* x, int64_t m,
                      double* lambda_out, const double* w, int32_t prec, void* ws,
                      size_t ws_bytes, void* stream) {
  if (m > 0 && lambda_out == nullptr) return FH_E_ARG;
  return eval_common(nodes, nullptr, n, d, x, m, nullptr, lambda_out, w, prec, ws, ws_bytes,
                     stream);
}

fh_status fh_lebesgue_max(const double* nodes, int64_t n, int32_t d, const double* w,
                          int32_t samples, int32_t rounds, double* lam_out, double* x_out,
                          double* best_out, int32_t prec, void* ws, size_t ws_bytes,
                          void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (samples < 1 || samples > 512 || rounds < 1 || rounds > 64) return FH_E_ARG;
  if (lam_out == nullptr && x_out == nullptr && best_out == nullptr) return FH_E_ARG;
  if (prec == FH_FP32_SPLIT) return FH_E_UNSUPPORTED;
  if (prec != FH_FP64) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, fh_workspace_size(FH_OP_LEBESGUE_MAX, n, 0, d, prec));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  LebesgueBufs b;
  layout_lebesgue_max(ws, n, &t, &b);
  hipError_t e = launch_pack(nodes, nullptr, w, n, d, t, false, static_cast<uint32_t*>(ws), s);
  if (e == hipSuccess)
    e = launch_lebesgue_max(t, n, samples, rounds, static_cast<uint32_t*>(ws) + 3, b,
                            lam_out ? lam_out : b.lam, x_out ? x_out : b.xk, best_out, s);
  return finish(e, ws, s);
}

size_t fh_multi_workspace_size(int64_t n, int32_t K) {
  if (n < 1 || n > FH_MAX_NODES || K < 1 || K > kMultiMax) return 0;
  MultiTable t;
  return layout_multi(nullptr, n, K, &t);
}

fh_status fh_eval_multi(const double* nodes, const double* values, int64_t n,
                        const int32_t* d_host, int32_t K, const double* x, int64_t m,
                        double* r_out, double* lambda_out, void* ws, size_t ws_bytes,
                        void* stream) {
  if (n < 1 || n > FH_MAX_NODES || nodes == nullptr || values == nullptr || d_host == nullptr)
    return FH_E_ARG;
  if (K < 1 || K > kMultiMax) return FH_E_ARG;
  if (m < 0 || (m > 0 && (x == nullptr || r_out == nullptr))) return FH_E_ARG;
  MultiDegrees deg{};
  bool shared = true;
  for (int32_t c = 0; c < K; ++c) {
    if (d_host[c] < 0 || (int64_t)d_host[c] > n - 1) return FH_E_DEGREE;
    deg.d[c] = d_host[c];
    shared = shared && d_host[c] == d_host[0];
  }
  fh_status st = check_ws(ws, ws_bytes, fh_multi_workspace_size(n, K));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  MultiTable t;
  layout_multi(ws, n, K, &t);
  return finish(launch_multi(nodes, values, n, deg, K, shared, x, m, t, r_out, lambda_out,
                             static_cast<uint32_t*>(ws), s),
                ws, s);
}

fh_status fh_eval_deriv(const double* nodes, const double* values, int64_t n, int32_t d,
                        const double* x, int64_t m, double* r_out, double* dr_out,
                        const double* w, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (values == nullptr || m < 0 || (m > 0 && (x == nullptr || dr_out == nullptr)))
    return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, eval_ws_min(n));
  if (st != FH_OK) return st;
  st = fh_prepare(nodes, values, n, d, w, prec, ws, ws_bytes, stream);
  if (st != FH_OK || m == 0) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  layout_tables(ws, n, &t);
  const hipError_t e =
      prec == FH_FP32_SPLIT
          ? launch_eval_deriv_split(x, m, t, n, static_cast<int32_t*>(ws) + 1, r_out, dr_out, s)
          : launch_eval_deriv(x, m, t, n, r_out, dr_out, s);
  return finish(e, ws, s);
}

fh_status fh_eval_backward(const double* nodes, const double* values, int64_t n, int32_t d,
                           const double* x, int64_t m, const double* grad_r, double* grad_values,
                           double* grad_x, double* grad_nodes, int32_t prec, void* ws,
                           size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (values == nullptr || m < 0 || (m > 0 && (x == nullptr || grad_r == nullptr)))
    return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, fh_workspace_size(FH_OP_BACKWARD, n, m, d, prec));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  BackwardBufs b;
  const bool split = prec == FH_FP32_SPLIT;
  layout_backward(ws, n, m, split, &t, &b);
  uint32_t* status = static_cast<uint32_t*>(ws);
  hipError_t e = launch_pack(nodes, values, nullptr, n, d, t, split, status, s);
  if (e == hipSuccess)
    e = launch_backward(nodes, x, grad_r, n, d, m, t, b, reinterpret_cast<int32_t*>(status) + 1,
                        grad_values, m > 0 ? grad_x : nullptr, grad_nodes, s);
  return finish(e, ws, s);
}

fh_status fh_eval_forward(const double* nodes, const double* values, int64_t n, int32_t d,
                          const double* x, int64_t m, double* r_out, double* dr_out,
                          int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (values == nullptr || m < 0 || (m > 0 && (x == nullptr || r_out == nullptr)))
    return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, fh_workspace_size(FH_OP_BACKWARD_SAVED, n, m, d, prec));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  BackwardBufs b;
  const bool split = prec == FH_FP32_SPLIT;
  layout_backward(ws, n, m, split, &t, &b, true);
  uint32_t* status = static_cast<uint32_t*>(ws);
  hipError_t e = launch_pack(nodes, values, nullptr, n, d, t, split, status, s);
  if (e == hipSuccess && m > 0) {
    if (split && dr_out) {
      e = launch_forward_saved_split(x, m, t, n, reinterpret_cast<int32_t*>(status) + 1, b,
                                     r_out, dr_out, s);
    } else if (split) {
      // as fh_eval_prepared chooses (the same r bits as fh_eval)
      const EvalConfig cfg = choose_eval_config(prec, n, 0, m, true, false);
      e = launch_eval_split(x, m, t, n, reinterpret_cast<int32_t*>(status) + 1, status + 3,
                            r_out, nullptr, cfg, s);
    } else {
      e = launch_forward_saved(x, m, t, n, b, r_out, dr_out, s);
    }
  } else if (e == hipSuccess && !split) {
    e = launch_forward_saved(x, 0, t, n, b, nullptr, nullptr, s);  // padding records only
  } else if (e == hipSuccess && dr_out) {
    e = launch_forward_saved_split(x, 0, t, n, reinterpret_cast<int32_t*>(status) + 1, b,
                                   nullptr, nullptr, s);
  }
  return finish(e, ws, s);
}

fh_status fh_eval_backward_saved(const double* nodes, int64_t n, int32_t d, const double* x,
                                 int64_t m, const double* dr, const double* grad_r,
                                 double* grad_values, double* grad_x, double* grad_nodes,
                                 int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  fh_status st = check_problem(nodes, n, d);
  if (st != FH_OK) return st;
  if (m < 0 || (m > 0 && (x == nullptr || grad_r == nullptr))) return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  st = check_ws(ws, ws_bytes, fh_workspace_size(FH_OP_BACKWARD_SAVED, n, m, d, prec));
  if (st != FH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  NodeTable t;
  BackwardBufs b;
  const bool split = prec == FH_FP32_SPLIT;
  layout_backward(ws, n, m, split, &t, &b, true);
  uint32_t* status = static_cast<uint32_t*>(ws);
  hipError_t e = hipSuccess;
  if (split && dr) {
    // the forward kept r' and the records for g = 1: dL/dx_p = g_p r'(x_p),
    // the node gradients from the records scaled by g and the node pass
    if (m > 0 && grad_x) e = launch_point_grad_from_derivative(grad_r, dr, m, grad_x, s);
    if (e == hipSuccess && (grad_values || grad_nodes)) {
      e = launch_backward_saved_split(grad_r, m, t, b, grad_nodes != nullptr, s);
      if (e == hipSuccess)
        e = launch_backward_tail(nodes, n, d, t, b, reinterpret_cast<int32_t*>(status) + 1,
                                 grad_values, grad_nodes, s);
    }
  } else if (split) {
    e = launch_backward(nodes, x, grad_r, n, d, m, t, b, reinterpret_cast<int32_t*>(status) + 1,
                        grad_values, m > 0 ? grad_x : nullptr, grad_nodes, s);
  } else {
    e = launch_backward_saved(nodes, x, dr, grad_r, n, d, m, t, b, grad_values, grad_x,
                              grad_nodes, s);
  }
  return finish(e, ws, s);
}

fh_status fh_device_status(void* ws, void* stream, uint32_t* bits_out) {
  if (ws == nullptr || bits_out == nullptr) return FH_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return FH_E_HIP;
  uint32_t bits = 0;
  if (hipMemcpy(&bits, ws, sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess) return FH_E_HIP;
  if (bits) {
    k_clear_word<<<1, 1, 0, s>>>(static_cast<uint32_t*>(ws));
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return FH_E_HIP;
  }
  *bits_out = bits;
  return status_from_bits(bits);
}

}  // extern "C"
