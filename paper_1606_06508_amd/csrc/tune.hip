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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>

#include "fh_internal.h"

namespace fhk {
namespace {

std::mutex g_mu;
int g_force[4] = {-1, -1, -1, -1};
std::unordered_map<int64_t, int> g_table;
bool g_cache_tried = false;

int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v && b < 62) ++b;
  return b;
}

// (family, ceil(log2 n_pad), ceil(log2 m)).  Whether Lambda is requested
// is not part of the key: the variant fixes the summation order, so r has
// the same bits with and without Lambda.
int64_t key(int32_t fam, int nb, int mb) { return ((int64_t)fam << 16) | (nb << 8) | mb; }

bool valid_family(int32_t fam) { return fam >= FH_FP64 && fam <= FH_TUNE_BATCHED_SPLIT; }

int variant_count(int32_t fam) {
  switch (fam) {
    case FH_FP64: return f64_variant_count();
    case FH_FP32_SPLIT: return split_variant_count();
    default: return batched_variant_count(fam == FH_TUNE_BATCHED_SPLIT);
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
  int32_t fam;
  int nb, mb;  // ceil(log2 n_pad), ceil(log2 m)
  int variant;
};
// (n = 1001: the single-call shape takes the variant of the nine-degree
// launch, 1 % slower than its own best, so both sum in the same order.)
constexpr Builtin kBuiltin[] = {
    {FH_FP64, 6, 14, 16},       {FH_FP64, 10, 20, 25},      {FH_FP64, 10, 24, 25},
    {FH_FP64, 12, 20, 21},      {FH_FP64, 13, 20, 21},      {FH_FP64, 13, 24, 25},
    {FH_FP32_SPLIT, 6, 14, 4},  {FH_FP32_SPLIT, 10, 20, 9}, {FH_FP32_SPLIT, 12, 20, 9},
    {FH_FP32_SPLIT, 13, 20, 9}, {FH_FP32_SPLIT, 13, 24, 9},
    // the 4096-instance batch (mean n 1041, 2.04e8 points)
    {FH_TUNE_BATCHED_FP64, 11, 28, 23}, {FH_TUNE_BATCHED_SPLIT, 11, 28, 5},
};

// Untuned shapes: two points per lane with the node range split over the
// four waves of a block and node blocks summed by node pairs (the tuner's
// choice for the large single-call shapes measured), four points per lane
// for the split form's small point sets; batches two points per lane.
int default_variant(int32_t fam, int nb, int mb) {
  for (const Builtin& b : kBuiltin)
    if (b.fam == fam && b.nb == nb && b.mb == mb) return b.variant;
  if (fam == FH_TUNE_BATCHED_FP64 || fam == FH_TUNE_BATCHED_SPLIT) return 1;
  if (fam == FH_FP32_SPLIT) return mb <= 16 ? 10 : 9;  // P = 4 / 2, quads, tile sums
  return 21;                                           // P = 2, S = 4, node pairs
}

int family_of(const char* name, size_t len) {
  static const char* kNames[4] = {"fp64", "split", "batched_fp64", "batched_split"};
  for (int f = 0; f < 4; ++f)
    if (std::strlen(kNames[f]) == len && std::strncmp(kNames[f], name, len) == 0) return f;
  if (len == 10 && std::strncmp(name, "fp32_split", 10) == 0) return FH_FP32_SPLIT;
  return -1;
}

// Value of "key" inside text[b, e): a number, or (str) a quoted string.
bool json_number(const std::string& t, size_t b, size_t e, const char* k, long long* v) {
  const std::string pat = std::string("\"") + k + "\"";
  const size_t at = t.find(pat, b);
  if (at == std::string::npos || at >= e) return false;
  size_t i = at + pat.size();
  while (i < e && (t[i] == ' ' || t[i] == ':' || t[i] == '\n' || t[i] == '\t')) ++i;
  char* end = nullptr;
  const long long x = std::strtoll(t.c_str() + i, &end, 10);
  if (end == t.c_str() + i) return false;
  *v = x;
  return true;
}

bool json_string(const std::string& t, size_t b, size_t e, const char* k, std::string* v) {
  const std::string pat = std::string("\"") + k + "\"";
  const size_t at = t.find(pat, b);
  if (at == std::string::npos || at >= e) return false;
  const size_t q0 = t.find('"', at + pat.size());
  if (q0 == std::string::npos || q0 >= e) return false;
  const size_t q1 = t.find('"', q0 + 1);
  if (q1 == std::string::npos || q1 >= e) return false;
  *v = t.substr(q0 + 1, q1 - q0 - 1);
  return true;
}

// FH_AUTOTUNE_CACHE: a table saved by the autotuner (JSON with "arch" and
// "entries" of {"precision", "n", "m", "variant", ...}), installed
// on first use if it was made on the current device's architecture.  Read
// once per process, with g_mu held.
void load_cache_locked() {
  if (g_cache_tried) return;
  g_cache_tried = true;
  const char* path = std::getenv("FH_AUTOTUNE_CACHE");
  if (path == nullptr || path[0] == 0) return;
  std::FILE* f = std::fopen(path, "rb");
  if (f == nullptr) {
    if (log_enabled()) std::fprintf(stderr, "[fh] FH_AUTOTUNE_CACHE: cannot open %s\n", path);
    return;
  }
  std::string t;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, got);
  std::fclose(f);
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch, have;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    have = prop.gcnArchName;
    have = have.substr(0, have.find(':'));
  }
  if (!json_string(t, 0, t.size(), "arch", &arch) || arch != have) {
    if (log_enabled())
      std::fprintf(stderr, "[fh] FH_AUTOTUNE_CACHE: %s made for '%s', device is '%s': ignored\n",
                   path, arch.c_str(), have.c_str());
    return;
  }
  size_t pos = t.find("\"entries\"");
  int installed = 0;
  while (pos != std::string::npos) {
    const size_t b = t.find('{', pos);
    if (b == std::string::npos) break;
    size_t e = b;
    for (int depth = 0; e < t.size(); ++e) {
      if (t[e] == '{') ++depth;
      if (t[e] == '}' && --depth == 0) break;
    }
    if (e >= t.size()) break;
    std::string prec;
    long long n = 0, m = 0, v = -1;
    if (json_string(t, b, e, "precision", &prec) && json_number(t, b, e, "n", &n) &&
        json_number(t, b, e, "m", &m) && json_number(t, b, e, "variant", &v)) {
      const int fam = family_of(prec.data(), prec.size());
      if (fam >= 0 && n >= 1 && m >= 1 && v >= 0 && v < variant_count(fam)) {
        g_table[key(fam, ceil_log2(round_up(n, kNodePad)), ceil_log2(m))] = (int)v;
        ++installed;
      }
    }
    pos = e + 1;
  }
  if (log_enabled())
    std::fprintf(stderr, "[fh] FH_AUTOTUNE_CACHE: %d entries installed from %s\n", installed,
                 path);
}

const char* family_name(int32_t fam) {
  static const char* kNames[4] = {"fp64", "split", "batched_fp64", "batched_split"};
  return valid_family(fam) ? kNames[fam] : "?";
}

}  // namespace

bool log_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("FH_LOG");
    return v && v[0] != 0 && v[0] != '0';
  }();
  return on;
}

EvalConfig choose_eval_config(int32_t prec, int64_t n, int32_t d, int64_t m, bool want_r,
                              bool want_l) {
  (void)d; (void)want_r; (void)want_l;
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  EvalConfig c;
  const char* source;
  const int64_t n_pad = round_up(n, kNodePad);
  const int nb = ceil_log2(n_pad), mb = ceil_log2(m);
  if (g_force[prec] >= 0) {
    c.variant = g_force[prec];
    source = "forced";
  } else {
    auto it = g_table.find(key(prec, nb, mb));
    if (it != g_table.end()) {
      c.variant = it->second;
      source = "tuned";
    } else {
      c.variant = default_variant(prec, nb, mb);
      source = "built-in";
    }
  }
  if (log_enabled()) {
    static std::unordered_set<int64_t> seen;
    const int64_t k = (key(prec, nb, mb) << 8) | c.variant;
    if (seen.insert(k).second)
      std::fprintf(stderr, "[fh] %s n=%lld m=%lld: variant %d (%s)\n", family_name(prec),
                   (long long)n, (long long)m, c.variant, source);
  }
  return c;
}

int bit_class(int32_t prec, int id) {
  if (prec == FH_FP64) {
    int p, g, s;
    f64_variant_shape(id, &p, &g, &s);
    return (f64_variant_octets(id) ? 1 << 25 : 0) | (f64_variant_pairs(id) ? 1 << 24 : 0) |
           (g << 16) | (s << 8) | f64_variant_block(id);
  }
  if (prec == FH_FP32_SPLIT) {
    int p, g, s;
    split_variant_shape(id, &p, &g, &s);
    return (g << 16) | split_variant_block(id);
  }
  return id;
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
  return batched_variant_block(id, prec == FH_TUNE_BATCHED_SPLIT);
}

int32_t fh_variant_node_pairs(int32_t prec, int32_t id) {
  if (!valid_family(prec) || id < 0 || id >= variant_count(prec)) return -1;
  if (prec == FH_FP64) return f64_variant_pairs(id) ? 1 : 0;
  return batched_variant_pairs(id, prec == FH_TUNE_BATCHED_SPLIT) ? 1 : 0;
}

int32_t fh_variant_octets(int32_t prec, int32_t id) {
  if (!valid_family(prec) || id < 0 || id >= variant_count(prec)) return -1;
  return prec == FH_FP64 && f64_variant_octets(id) ? 1 : 0;
}

int64_t fh_variant_strip_points(int32_t prec, int32_t id) {
  if (!valid_family(prec) || id < 0 || id >= variant_count(prec)) return -1;
  int p, g, s;
  shape(prec, id, &p, &g, &s);
  if (prec == FH_FP64) return 64LL * p * (4 / s);
  if (prec == FH_FP32_SPLIT) return 256LL * p;
  return batched_variant_strip(id, prec == FH_TUNE_BATCHED_SPLIT);
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
  load_cache_locked();
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
