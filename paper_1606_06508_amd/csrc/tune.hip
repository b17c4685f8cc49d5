// Kernel-variant selection for the evaluation kernels.
//
// Each evaluation kernel comes in a table of variants (points per lane,
// node group, node split; see eval_f64.hip / eval_split.hip).  The variant
// for a call is looked up by (precision, ceil(log2 n_pad), ceil(log2 m)) in
// a per-process table that the autotuner fills (fh_tune_set, driven by
// paper_1606_06508_amd/autotune.py, which times every variant on the shape
// and keeps the fastest).  Shapes nobody tuned at run time use the built-in
// table below (the tuner's choices on MI355X) or a size rule; fh_tune_force
// pins one variant for all shapes (used by the tuner while it measures).
#include <mutex>
#include <unordered_map>

#include "fh_internal.h"

namespace fhk {
namespace {

std::mutex g_mu;
int g_force[4] = {-1, -1, -1, -1};
std::unordered_map<int64_t, int> g_table;

int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v && b < 62) ++b;
  return b;
}

int64_t key(int32_t prec, int nb, int mb) { return ((int64_t)prec << 16) | (nb << 8) | mb; }

bool valid_family(int32_t fam) { return fam >= FH_FP64 && fam <= FH_TUNE_BATCHED_SPLIT; }

int variant_count(int32_t fam) {
  switch (fam) {
    case FH_FP64: return f64_variant_count();
    case FH_FP32_SPLIT: return split_variant_count();
    default: return batched_variant_count();
  }
}

void shape(int32_t fam, int id, int* p, int* g, int* s) {
  switch (fam) {
    case FH_FP64: f64_variant_shape(id, p, g, s); return;
    case FH_FP32_SPLIT: split_variant_shape(id, p, g, s); return;
    default: batched_variant_shape(id, p, g, s, fam == FH_TUNE_BATCHED_SPLIT);
  }
}

// Built-in table: the autotuner's choices measured on MI355X (gfx950) for
// the shapes of the evaluation study, keyed like the run-time table.
struct Builtin {
  int32_t prec;
  int nb, mb;  // ceil(log2 n_pad), ceil(log2 m)
  int variant;
};
constexpr Builtin kBuiltin[] = {
    {FH_FP64, 6, 14, 7},       {FH_FP64, 10, 20, 17},      {FH_FP64, 10, 24, 18},
    {FH_FP64, 12, 20, 16},
    {FH_FP64, 13, 20, 16},     {FH_FP64, 13, 24, 18},      {FH_FP32_SPLIT, 6, 14, 4},
    {FH_FP32_SPLIT, 10, 20, 9}, {FH_FP32_SPLIT, 12, 20, 9}, {FH_FP32_SPLIT, 13, 20, 9},
    {FH_FP32_SPLIT, 13, 24, 9},
};

// Untuned shapes: two points per lane with the node range split over the
// four waves of a block and the Lebesgue sum taken by node blocks (the
// tuner's choice for every large shape measured), four points per lane for
// the split form's small point sets.
int default_variant(int32_t prec, int nb, int mb) {
  for (const Builtin& b : kBuiltin)
    if (b.prec == prec && b.nb == nb && b.mb == mb) return b.variant;
  if (prec == FH_TUNE_BATCHED_FP64 || prec == FH_TUNE_BATCHED_SPLIT) return 1;  // P = 2
  if (prec == FH_FP32_SPLIT) return mb <= 16 ? 10 : 9;  // P = 4 / 2, quads, tile sums
  return 16;                                            // P = 2, G = 8, S = 4, U = 16
}

}  // namespace

EvalConfig choose_eval_config(int32_t prec, int64_t n, int32_t d, int64_t m, bool want_r,
                              bool want_l) {
  (void)d; (void)want_r; (void)want_l;
  std::lock_guard<std::mutex> lk(g_mu);
  EvalConfig c;
  if (g_force[prec] >= 0) {
    c.variant = g_force[prec];
    return c;
  }
  const int64_t n_pad = round_up(n, kNodePad);
  const int nb = ceil_log2(n_pad), mb = ceil_log2(m);
  auto it = g_table.find(key(prec, nb, mb));
  c.variant = it != g_table.end() ? it->second : default_variant(prec, nb, mb);
  return c;
}

}  // namespace fhk

using namespace fhk;

extern "C" {

int32_t fh_variant_count(int32_t prec) {
  if (!valid_family(prec)) return 0;
  return variant_count(prec);
}

fh_status fh_variant_shape(int32_t prec, int32_t id, int32_t* points_per_lane, int32_t* group,
                           int32_t* node_split) {
  if (!valid_family(prec)) return FH_E_ARG;
  if (id < 0 || id >= variant_count(prec) || !points_per_lane || !group || !node_split)
    return FH_E_ARG;
  int p, g, s;
  shape(prec, id, &p, &g, &s);
  *points_per_lane = p;
  *group = g;
  *node_split = s;
  return FH_OK;
}

int32_t fh_variant_lebesgue_block(int32_t prec, int32_t id) {
  if (!valid_family(prec) || id < 0 || id >= variant_count(prec)) return -1;
  if (prec == FH_FP64) return f64_variant_block(id);
  if (prec == FH_FP32_SPLIT) return split_variant_block(id);
  // batches: split by tiles (library weights), binary64 plain
  return prec == FH_TUNE_BATCHED_FP64 ? 0 : 32;
}

fh_status fh_tune_force(int32_t prec, int32_t id) {
  if (!valid_family(prec)) return FH_E_ARG;
  if (id < -1 || id >= variant_count(prec)) return FH_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_force[prec] = id;
  return FH_OK;
}

fh_status fh_tune_set(int32_t prec, int64_t n, int64_t m, int32_t id) {
  if (!valid_family(prec)) return FH_E_ARG;
  if (n < 1 || m < 1 || id < -1 || id >= variant_count(prec)) return FH_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t k = key(prec, ceil_log2(round_up(n, kNodePad)), ceil_log2(m));
  if (id < 0)
    g_table.erase(k);
  else
    g_table[k] = id;
  return FH_OK;
}

int32_t fh_tune_get(int32_t prec, int64_t n, int64_t m) {
  if (!valid_family(prec)) return -1;
  if (n < 1 || m < 1) return -1;
  return choose_eval_config(prec, n, 0, m, true, true).variant;
}

}  // extern "C"
