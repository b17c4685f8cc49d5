// Internal declarations of libfh (HIP, gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fh.h"
#include "bwd_math.h"

namespace fhk {

// The first kStatusBytes of every workspace: word 0 = sticky status bits,
// word 1 = binary32 weight scaling exponent e of the split form
// (max|w| = m 2^e, 1/2 <= m < 1), word 2 = ef - e with 2^ef the scale of
// the weighted values w f (split_table_scale), word 3 = 1 if the node
// table's weights alternate strictly in sign (always for the library's
// weights; caller weights are checked pair by pair), written by every
// packing; word 4 = 1 if a split table is too ill-conditioned for binary32
// terms (split_table_wide, written by the split packing); words 5..
// reserved.
constexpr size_t kStatusBytes = 256;
// Node tables are padded to a multiple of this many records; padding
// records repeat the last node with zero weight, so they add nothing.
constexpr int64_t kNodePad = 64;
constexpr size_t kAlign = 256;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline size_t align_up(size_t a) { return (a + kAlign - 1) / kAlign * kAlign; }

// Node table of one interpolant in structure-of-arrays form (device).
struct NodeTable {
  double* x;      // [n_pad] x_k
  double* w;      // [n_pad] w_k
  double* wf;     // [n_pad] w_k * f_k
  double* f;      // [n_pad] f_k (exact-hit branch)
  float4* s;      // [n_pad] split form: {binary32 head of x_k, binary32 tail
                  // x_k - head, binary32 of w_k 2^-e, binary32 of w_k f_k 2^-ef}
  double* pr;     // [n_pad / kPairBlock][kPairRec] node-pair records (binary64)
  uint32_t* pok;  // [ceil(n_pad / 256)] bit i of word w: pair block 16 w + i passed
                  // the pack's test (or lies beyond the nodes)
  int64_t n_pad;
};

// Workspace layout of FH_OP_EVAL / FH_OP_BACKWARD (node tables after the
// status block).  Returns bytes used.
size_t layout_tables(void* ws, int64_t n, NodeTable* t);

// Octet launch variants (binary64): the table's octet records and summary
// word (pair_math.h, written by launch_octet_records) and the original
// position of each sorted point (order[i]: where sorted point i came from,
// written by launch_sort_points).  The other variants ignore it.
struct OctetArgs {
  const double* rec;
  const uint32_t* ok;
  const int32_t* order;
};

// Launch configuration of an evaluation kernel: an index into the kernel's
// variant table (points per lane, node group, node split), chosen per
// problem shape by the tuner (tune.hip).
struct EvalConfig {
  int variant;
};
EvalConfig choose_eval_config(int32_t prec, int64_t n, int32_t d, int64_t m, bool want_r,
                              bool want_l);
int f64_variant_count();
void f64_variant_shape(int id, int* p, int* g, int* s);
int f64_variant_block(int id);  // Lebesgue block length U, 0 for plain sums
bool f64_variant_pairs(int id);  // sums by node pairs (pair_math.h)
bool f64_variant_octets(int id);  // pairs, and octets for the blocks far from the points
int f64_variant_octet_twin(int id);  // the pair variant of the same shape
int split_variant_count();
void split_variant_shape(int id, int* p, int* g, int* s);
int split_variant_block(int id);  // node tile of the block sums, 0 for plain sums
int batched_variant_count(bool split);
void batched_variant_shape(int id, int* p, int* g, int* s, bool split);
int batched_variant_block(int id, bool split);      // Lebesgue block / node tile, 0 for plain
bool batched_variant_pairs(int id, bool split);     // binary64 sums by node pairs
int64_t batched_variant_strip(int id, bool split);  // points of one work item
// Variants of one family with the same bit class give the same bits for the
// same point and table (they differ only in points per lane or strip length).
int bit_class(int32_t prec, int id);
// FH_LOG set (and not "0"): launch choices are reported on stderr.
bool log_enabled();

// Adjoint: points are processed in `chunks` chunks of `chunk` points
// (m_pad = chunks * chunk, the tail padded with neutral records) so that the
// per-node pass has enough (node tile, chunk) waves.
struct BackwardPlan {
  int64_t n_pad, chunk, chunks, m_pad;
  int p;       // points per lane in the per-point pass (binary64)
  int q;       // nodes per lane in the per-node pass
  int g;       // points per simultaneous inversion in the per-node pass (binary64)
  int groups;  // saved-state adjoint: node tile groups of the fused pass (0: not planned)
  bool split;  // precision-split passes 1 and 2
};
// At most this many node tile groups in the saved-state adjoint's fused pass
// (its point-side partial sums take groups * m_pad doubles).
constexpr int32_t kMaxTileGroups = 64;
struct BackwardBufs {
  BackwardPlan plan;
  PointRecs rec;  // per-point records of pass 1 (five [m_pad] arrays)
  float4* rec32;  // [m_pad] binary32 point records (split only, else null)
  double* part;   // [chunks][6][n_pad] per-chunk node sums
  double* sums;   // [6][n_pad] node sums over all chunks
  double* dw;     // [n_pad] dL/dw_k
  double* dxd;    // [n_pad] direct dL/dx_k at fixed weights
  // saved-state adjoint (FH_OP_BACKWARD_SAVED) only, else null:
  PointRecs saved;  // the forward's records for g = 1: {x (= rec.x), 1/D, r,
                    // 1 at a hit, r'(x_j) at a hit} (split: 2^e / D)
  double* gpart;    // [groups][m_pad] point-side sums per node tile group (binary64)
  float4* saved32;  // [m_pad] {head, tail, binary64-path flag, 0} (split)
};
// saved: plan the saved-state adjoint (binary64 only; split plans ignore it).
BackwardPlan plan_backward(int64_t n, int64_t m, bool split, bool saved = false);
// Workspace layout of FH_OP_BACKWARD, or of FH_OP_BACKWARD_SAVED when saved
// (node tables, then the buffers above).
size_t layout_backward(void* ws, int64_t n, int64_t m, bool split, NodeTable* t,
                       BackwardBufs* b, bool saved = false);

// Several interpolants on the same nodes and points (fh_eval_multi).
constexpr int kMultiMax = 64;
struct MultiDegrees {
  int32_t d[kMultiMax];
};
// Node tables of K columns (plus zero padding): x[n_pad] shared;
// w[.][n_pad] (only row 0 used when every column has the same degree),
// wf[.][n_pad] = w f, f[.][n_pad].
struct MultiTable {
  double *x, *w, *wf, *f;
  int64_t n_pad;
};
size_t layout_multi(void* ws, int64_t n, int32_t K, MultiTable* t);
// Columns the tables hold: K plus zero padding up to a whole number of
// launch chunks.
int64_t multi_padded_columns(int32_t K);
// Packs the K tables, then evaluates r (and Lambda if lam) of every column:
// r[c * m + p], lam[c * m + p].
hipError_t launch_multi(const double* nodes, const double* values, int64_t n,
                        const MultiDegrees& deg, int32_t K, bool shared, const double* x,
                        int64_t m, const MultiTable& t, double* r, double* lam, uint32_t* status,
                        hipStream_t s);

// ---- launchers (each returns the launch error, hipSuccess on success) ----
hipError_t launch_weights(const double* nodes, int64_t n, int32_t d, double* w_out,
                          uint32_t* status, hipStream_t s);
// Tables of up to kPackMany degrees of one interpolant (FP64), one launch.
constexpr int kPackMany = 16;
struct PackMany {
  double* x[kPackMany];
  double* w[kPackMany];
  double* wf[kPackMany];
  double* f[kPackMany];
  double* pr[kPackMany];
  uint32_t* pok[kPackMany];
  uint32_t* status[kPackMany];
  int32_t d[kPackMany];
};
hipError_t launch_pack_many(const double* nodes, const double* values, int64_t n,
                            const PackMany& a, int32_t K, hipStream_t s);
hipError_t launch_pack(const double* nodes, const double* values, const double* w_in, int64_t n,
                       int32_t d, const NodeTable& t, bool split, uint32_t* status,
                       hipStream_t s);
// Up to kEvalMany prepared binary64 tables with the same node count,
// evaluated on the same points in one launch (grid.y = table).
constexpr int kEvalMany = 16;
struct EvalMany {
  const double* x[kEvalMany];
  const double* w[kEvalMany];
  const double* wf[kEvalMany];
  const double* f[kEvalMany];
  const double* pr[kEvalMany];
  const uint32_t* pok[kEvalMany];
  const uint32_t* alt[kEvalMany];
  double* r[kEvalMany];
  double* lam[kEvalMany];
  const double* oc[kEvalMany];    // octet variants: each table's octet records
  const uint32_t* ook[kEvalMany];  // and summary word
  const int32_t* order;            // original positions of the sorted points
};
// The octet variants' buffers in an evaluation workspace, after the node
// tables: the table's octet records ([n_pad / kPairBlock][kOctetEvalRec])
// and summary word, and room for m points sorted by node block (per tile
// of the sort its count, then sorted start, per block; each point's block;
// the sorted points and their original positions; a launch over several
// tables sorts into its first table's workspace).
struct OctetBufs {
  double* rec;
  uint32_t* ok;
  int32_t* hist;
  int32_t* key;
  double* xs;
  int32_t* order;
};
// Returns the bytes of an evaluation workspace with room for m sorted
// points (the size fh_workspace_size reports for FH_OP_EVAL in binary64).
size_t layout_octets(void* ws, int64_t n, int64_t m, OctetBufs* b);
// Whether the octet variants serve n nodes and m points at all.
bool octets_possible(int64_t n, int64_t m);
// Octet records and summary words of K tables of n nodes (one workgroup
// each).
struct OctetTables {
  const double* x[kEvalMany];
  const double* w[kEvalMany];
  const double* wf[kEvalMany];
  double* rec[kEvalMany];
  uint32_t* ok[kEvalMany];
};
hipError_t launch_octet_records(const OctetTables& a, int32_t K, int64_t n, int64_t n_pad,
                                hipStream_t s);
// The m points x sorted by node block of the table tx into b.xs, with their
// original positions in b.order.
hipError_t launch_sort_points(const double* x, int64_t m, const double* tx, int64_t n_pad,
                              const OctetBufs& b, hipStream_t s);
// r / lam: whether every table's r / Lambda is written.
hipError_t launch_eval_f64_many(const double* x, int64_t m, int64_t n, int64_t n_pad,
                                const EvalMany& a, int32_t K, bool r, bool lam,
                                const EvalConfig& cfg, hipStream_t s);
// alt: status word 3 of the workspace (1 if the table's weights alternate
// in sign, written by launch_pack), read by the Lebesgue-block variants.
// Octet variants: x are the points sorted by launch_sort_points and oa
// names the table's octet records and the points' original positions.
hipError_t launch_eval_f64(const double* x, int64_t m, const NodeTable& t, int64_t n,
                           const uint32_t* alt, double* r, double* lam, const EvalConfig& cfg,
                           const OctetArgs& oa, hipStream_t s);
// scale_exp: the split scaling exponent (status word 1) when b.plan.split.
hipError_t launch_backward(const double* nodes, const double* x, const double* g, int64_t n,
                           int32_t d, int64_t m, const NodeTable& t, const BackwardBufs& b,
                           const int32_t* scale_exp, double* df, double* dx, double* dxn,
                           hipStream_t s);
// Saved-state adjoint (binary64): the forward writes r and b.saved; the
// backward scales the saved records by g and runs one fused pass over the
// (point, node) pairs for the node sums and dL/dx_p together.
// dr (nullable): the forward also writes r'(x_p) there (E and F summed too),
// and the backward then takes dL/dx_p = g_p r'(x_p) from it.
hipError_t launch_forward_saved(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                const BackwardBufs& b, double* r, double* dr, hipStream_t s);
hipError_t launch_backward_saved(const double* nodes, const double* x, const double* dr,
                                 const double* g, int64_t n, int32_t d, int64_t m,
                                 const NodeTable& t, const BackwardBufs& b, double* df,
                                 double* dx, double* dxn, hipStream_t s);
// Split saved state (prec FH_FP32_SPLIT, forward with r'): the split point
// pass for g = 1 writes r, r' and b.saved / b.saved32; the backward scales
// them by g into b.rec / b.rec32 and runs the split node pass (full: all
// four sums).
hipError_t launch_forward_saved_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                      const int32_t* scale, const BackwardBufs& b, double* r,
                                      double* dr, hipStream_t s);
hipError_t launch_backward_saved_split(const double* g, int64_t m, const NodeTable& t,
                                       const BackwardBufs& b, bool full, hipStream_t s);
// Passes 3 and 4 of the adjoint (chunk reduction, per-node finish, weight
// chain) from the chunk partials in b.part; scale_exp: the split scaling
// exponent (null for binary64).
hipError_t launch_backward_tail(const double* nodes, int64_t n, int32_t d, const NodeTable& t,
                                const BackwardBufs& b, const int32_t* scale_exp, double* df,
                                double* dxn, hipStream_t s);
// dx[p] = g[p] dr[p] for p < m.
hipError_t launch_point_grad_from_derivative(const double* g, const double* dr, int64_t m,
                                             double* dx, hipStream_t s);
// The per-node split kernel for q nodes per lane (occupancy queries).
const void* bwd_nodes_split_kernel(int q);
// nodes_pass: run the per-node pass (dL/df or the node gradient wanted);
// full: all four sums there (the node gradient wanted), else S1 only.
hipError_t launch_backward_split_passes(const double* x, const double* g, int64_t n, int64_t m,
                                        const NodeTable& t, const BackwardBufs& b,
                                        const int32_t* scale_exp, double* dx, bool nodes_pass,
                                        bool full, hipStream_t s);
// scale: status words 1.. of the workspace (e, ef - e) written by the packing.
// r and r' at m points from a packed node table (binary64 / split).
hipError_t launch_eval_deriv(const double* x, int64_t m, const NodeTable& t, int64_t n, double* r,
                             double* dr, hipStream_t s);
hipError_t launch_eval_deriv_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                                   const int32_t* scale, double* r, double* dr, hipStream_t s);
// Workspace of FH_OP_LEBESGUE_MAX beyond the node tables: per-interval
// maxima and their locations ([n-1] each), the octet records of the node
// blocks (written by the search's own packing) and their summary word.
struct LebesgueBufs {
  double* lam;
  double* xk;
  double* oct;
  uint32_t* oct_ok;
};
// Workspace layout of FH_OP_LEBESGUE_MAX: node tables, then LebesgueBufs.
// Returns bytes used.
size_t layout_lebesgue_max(void* ws, int64_t n, NodeTable* t, LebesgueBufs* bufs);
// Per-interval maxima of Lambda (lam, xk: [n-1], not null) by the grid zoom
// of `rounds` rounds of `samples` samples; best (if not null) = {the
// constant, its location}; alt: status word 3 (weights alternate in sign);
// bufs: octet records and summary word, written here first.
hipError_t launch_lebesgue_max(const NodeTable& t, int64_t n, int32_t samples, int32_t rounds,
                               const uint32_t* alt, const LebesgueBufs& bufs, double* lam,
                               double* xk, double* best, hipStream_t s);
hipError_t launch_eval_split(const double* x, int64_t m, const NodeTable& t, int64_t n,
                             const int32_t* scale, const uint32_t* alt, double* r, double* lam,
                             const EvalConfig& cfg, hipStream_t s);

}  // namespace fhk
