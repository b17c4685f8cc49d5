/*
 * fh.h -- C ABI of the MI355X (gfx950) Floater-Hormann interpolation library
 * (libfh.so).
 *
 * The library evaluates linear barycentric rational interpolants of the
 * Floater-Hormann family (M. S. Floater, K. Hormann, "Barycentric rational
 * interpolation with no poles and high rates of approximation", Numer. Math.
 * 107, 2007):
 *
 *   nodes x_0 < x_1 < ... < x_{n-1}, data f_k, blending degree 0 <= d <= n-1,
 *   weights  w_k = sum_{i in J_k} (-1)^i prod_{j=i..i+d, j!=k} 1/(x_k - x_j),
 *            J_k = { i : max(0, k-d) <= i <= min(k, n-1-d) },
 *   value    r(x) = sum_k a_k(x) f_k / sum_k a_k(x),   a_k(x) = w_k / (x - x_k),
 *   Lebesgue Lambda(x) = sum_k |a_k(x)| / |sum_k a_k(x)|,
 *   exact hit x == x_j (binary64 equality): r = f_j bit-for-bit, Lambda = 1.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Every array argument is a DEVICE pointer (HBM of the current HIP
 *    device), owned by the caller.  The library never frees, retains or
 *    reallocates caller memory (except that an fh_batch keeps the pointers
 *    it was created with, see below).
 *  - Arrays are dense, contiguous binary64 unless stated otherwise.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Every call only enqueues work on `stream` and returns; results are
 *    valid once the stream has reached that point.
 *  - `ws` / `ws_bytes` is a caller-owned device workspace of at least
 *    fh_workspace_size(op, n, m, d, prec) bytes, 256-byte aligned.  Its first
 *    256 bytes hold the device status word (sticky error bits, see
 *    fh_device_status); they must be zero before the first use of a
 *    workspace (allocate it zeroed).  Calls that share a workspace must be
 *    ordered (same stream); concurrent calls need separate workspaces.
 *  - Host-checkable errors are returned synchronously and no work is
 *    enqueued: FH_E_ARG (n < 1 or n > FH_MAX_NODES, m < 0, a NULL pointer
 *    that is needed -- point and output arrays are needed only when m > 0 --
 *    a bad precision or op code), FH_E_DEGREE (d < 0 or d > n-1), FH_E_WORKSPACE
 *    (workspace missing, too small or misaligned).
 *  - Properties of the node VALUES (strictly increasing, finite, weights
 *    representable) are checked on the device.  A violation sets bits in the
 *    workspace status word; the outputs are then unspecified.  The bits are
 *    read back by fh_device_status; with the environment variable
 *    FH_SYNC_CHECK=1 every call synchronizes and returns them as a status.
 *  - NaN conventions (the paper's scaling algorithms propagate NaNs; the same
 *    rule here): a NaN point gives r = Lambda = NaN; a NaN value f_k gives NaN
 *    at every point except exact hits on other nodes; an infinite point makes
 *    every a_k zero, hence r = 0/0 = NaN.
 *  - Results are specified for points whose distance to every node is either
 *    zero (a hit) or at least 2^-250 times the node span; closer points may
 *    give non-finite results, as they do in binary64 arithmetic by the
 *    definition itself (w_k / (x - x_k) overflows).
 *
 * Precision
 *  - FH_FP64: every step in binary64.
 *  - FH_FP32_SPLIT: weights, the differences x - x_k and the final quotient
 *    in binary64; the reciprocals and the O(m*n) sums in binary32, with
 *    per-tile binary32 partial sums promoted into binary64 accumulators.  The
 *    weights are scaled by an exact power of two 2^-e (e = exponent of
 *    max|w_k|) before rounding to binary32, which changes neither r nor
 *    Lambda (the paper's key idea of scaling by powers of the base, exact by
 *    its rounding fact (rndA)).
 */
#ifndef FH_H
#define FH_H

#include <stddef.h>
#include <stdint.h>

/* Largest node count of one interpolant (2^28): node tables and node loops
 * index with 32-bit integers, and a larger n is refused with FH_E_ARG. */
#define FH_MAX_NODES (1LL << 28)

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FH_OK = 0,
  FH_E_ARG = 1,         /* bad size, NULL pointer, bad enum value               */
  FH_E_DEGREE = 2,      /* d < 0 or d > n-1                                      */
  FH_E_NODES = 3,       /* (device) nodes not strictly increasing               */
  FH_E_NONFINITE = 4,   /* (device) a node is NaN or infinite                   */
  FH_E_RANGE = 5,       /* (device) a weight product under/overflowed          */
  FH_E_WORKSPACE = 6,   /* workspace NULL, too small or not 256-byte aligned    */
  FH_E_HIP = 7,         /* a HIP runtime call failed                            */
  FH_E_UNSUPPORTED = 8, /* combination the library does not provide              */
  FH_E_TOO_LARGE = 9    /* problem exceeds the fixed scratch of fh_eval_noalloc */
} fh_status;

typedef enum { FH_FP64 = 0, FH_FP32_SPLIT = 1 } fh_precision;

/* Operation codes for fh_workspace_size. */
typedef enum {
  FH_OP_WEIGHTS = 0,
  FH_OP_EVAL = 1,       /* also fh_lebesgue */
  FH_OP_BACKWARD = 2,
  FH_OP_LEBESGUE_MAX = 3, /* fh_lebesgue_max (m ignored) */
  FH_OP_BACKWARD_SAVED = 4 /* fh_eval_forward + fh_eval_backward_saved */
} fh_op;

/* Device status bits (fh_device_status). */
#define FH_FLAG_NODES 0x1u     /* some x_k >= x_{k+1}                  */
#define FH_FLAG_NONFINITE 0x2u /* some x_k is NaN or infinite          */
#define FH_FLAG_RANGE 0x4u     /* a weight product is zero, subnormal or infinite */

/* Bytes of workspace an operation needs (0 on bad arguments).  `m` is the
 * number of evaluation points; for FH_OP_WEIGHTS it is ignored.  For
 * FH_OP_EVAL in binary64 the size includes, beyond the node tables, the
 * octet records and room for m points sorted by node block, which the
 * octet launch variants use (fh_variant_octets).  The evaluation calls
 * check only for the node tables; with fh_workspace_size(FH_OP_EVAL, n, m,
 * d, prec) bytes they can run the octet variants for up to m points, and
 * with less room they run the pair variant of the same shape. */
size_t fh_workspace_size(int32_t op, int64_t n, int64_t m, int32_t d, int32_t prec);

/* Node weights w_k of the definition above (Floater & Hormann 2007, the
 * barycentric form and its weights).  O(n d^2) work, one thread per node.
 * Every product is formed in ascending j, inverted with one IEEE division,
 * signed by (-1)^i and added in ascending i without FMA contraction, so the
 * result is reproducible bit-for-bit.
 *   nodes  [n]  strictly increasing abscissae x_k
 *   d           blending degree, 0 <= d <= n-1
 *   w_out  [n]  weights (unscaled)
 *   ws          workspace (FH_OP_WEIGHTS): status word only            */
fh_status fh_weights(const double* nodes, int64_t n, int32_t d, double* w_out, void* ws,
                     size_t ws_bytes, void* stream);

/* r(x_p) (and optionally Lambda(x_p)) at m points: the weight pass (unless
 * `w` is given) followed by the fused second-form sum N = sum a_k f_k,
 * D = sum a_k, L = sum |a_k| and the quotient, with the exact-hit branch.
 *   nodes, values [n]   x_k and f_k
 *   x          [m]      evaluation points (any order, any values)
 *   r_out      [m]      r(x_p)
 *   lambda_out [m]      Lambda(x_p), or NULL to skip the Lebesgue sum
 *   w          [n]      weights from fh_weights, or NULL to compute them here
 *   prec                FH_FP64 or FH_FP32_SPLIT
 *   ws                  workspace of fh_workspace_size(FH_OP_EVAL, ...)   */
fh_status fh_eval(const double* nodes, const double* values, int64_t n, int32_t d,
                  const double* x, int64_t m, double* r_out, double* lambda_out, const double* w,
                  int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* fh_eval for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, results and bits are those of fh_eval, but there is no `ws`:
 * the node table lives in a fixed device array of FH_NOALLOC_SCRATCH_BYTES
 * bytes inside the library, one per GPU, held until the process ends (its
 * device address is resolved on the first call on each device).  Nothing
 * is allocated, on the device or through any library, in any call.
 *   n              at most FH_NOALLOC_MAX_NODES (the largest table the array
 *                  holds); a larger n returns FH_E_TOO_LARGE, before any
 *                  work is enqueued
 *   other errors   as in fh_eval (FH_E_HIP if the array's address cannot be
 *                  resolved)
 * Every call on one GPU uses that GPU's one array, and the array keeps the
 * last call's table: calls that overlap on one GPU (different streams or
 * host threads without ordering) race and give undefined results; order
 * them on one stream.  Each call clears the array's status block first, so
 * device-side node checks report only under FH_SYNC_CHECK=1 (no workspace
 * is exposed to read them back later). */
#define FH_NOALLOC_SCRATCH_BYTES ((size_t)2 << 20)
#define FH_NOALLOC_MAX_NODES 28288LL
fh_status fh_eval_noalloc(const double* nodes, const double* values, int64_t n, int32_t d,
                          const double* x, int64_t m, double* r_out, double* lambda_out,
                          const double* w, int32_t prec, void* stream);

/* Two-phase form of fh_eval for evaluating one interpolant on many point
 * batches.  fh_prepare runs the weight pass (unless `w` is given) and packs
 * the node table (x_k, w_k, w_k f_k, f_k; binary32 copies for
 * FH_FP32_SPLIT) into `ws`; fh_eval_prepared then runs only the evaluation
 * kernel against that table.  `n` and `prec` must repeat the fh_prepare
 * call, and the table must not be overwritten in between.  A table prepared
 * with values == NULL supports lambda_out only (r_out must be NULL).
 * fh_eval(...) is exactly fh_prepare(...) followed by fh_eval_prepared(...). */
fh_status fh_prepare(const double* nodes, const double* values, int64_t n, int32_t d,
                     const double* w, int32_t prec, void* ws, size_t ws_bytes, void* stream);
fh_status fh_eval_prepared(void* ws, size_t ws_bytes, int64_t n, int32_t prec, const double* x,
                           int64_t m, double* r_out, double* lambda_out, void* stream);

/* fh_prepare for K degrees of one interpolant at once (a sweep over d), in
 * one launch: workspace ws_host[c] gets the table of degree d_host[c], the
 * same bits fh_prepare(nodes, values, n, d_host[c], NULL, prec, ws_host[c],
 * ...) writes; each is then evaluated with fh_eval_prepared.
 *   d_host   host array of K degrees, each in 0..n-1;  1 <= K <= 16
 *   ws_host  host array of K distinct device workspaces, each of at least
 *            fh_workspace_size(FH_OP_EVAL, n, m, d_host[c], prec) <= ws_bytes
 *            bytes (the same ws_bytes is checked for all)
 *   prec     FH_FP64 (FH_FP32_SPLIT tables: FH_E_UNSUPPORTED; use fh_prepare)
 *   values   may be NULL (tables for Lambda only, as with fh_prepare)
 * Errors as in fh_prepare; FH_E_ARG also for K out of range or a workspace
 * listed twice.  The library's weights are computed, never caller weights. */
fh_status fh_prepare_many(const double* nodes, const double* values, int64_t n,
                          const int32_t* d_host, int32_t K, int32_t prec, void* const* ws_host,
                          size_t ws_bytes, void* stream);

/* fh_eval_prepared for K prepared tables with the same node count n on the
 * same points, in one launch (for instance the degrees of a sweep prepared
 * by fh_prepare_many): table c writes r_host[c][0..m) and
 * lambda_host[c][0..m), the bits fh_eval_prepared(ws_host[c], ...) writes
 * for the same m: the launch takes the variant tuned for its K * m points
 * only when that variant sums in the same order as the one a single call
 * with m points would take (they differ only in points per lane), and that
 * single call's variant otherwise.  One launch instead of K saves, per
 * table, the drain of the launch's last blocks and the gap before the next
 * launch.
 *   ws_host      host array of K device workspaces prepared in binary64
 *                with n nodes (fh_prepare or fh_prepare_many), each of at
 *                least fh_workspace_size(FH_OP_EVAL, n, m, 0, prec) <=
 *                ws_bytes bytes;  1 <= K <= 16
 *   r_host       host array of K device output pointers (m doubles each),
 *                or NULL for no r; lambda_host likewise for Lambda; not
 *                both NULL, and no NULL entry in an array that is given
 *   prec         FH_FP64 (FH_FP32_SPLIT: FH_E_UNSUPPORTED)
 * Outputs of different tables must not overlap.  Errors as in
 * fh_eval_prepared; FH_E_ARG also for K out of range. */
fh_status fh_eval_prepared_many(void* const* ws_host, size_t ws_bytes, int32_t K, int64_t n,
                                int32_t prec, const double* x, int64_t m, double* const* r_host,
                                double* const* lambda_host, void* stream);

/* Lambda(x_p) only (the Lebesgue function of the interpolation scheme,
 * sum_k |b_k(x)| with cardinal functions b_k = a_k / sum_j a_j).  Arguments
 * as in fh_eval; no values are needed. */
fh_status fh_lebesgue(const double* nodes, int64_t n, int32_t d, const double* x, int64_t m,
                      double* lambda_out, const double* w, int32_t prec, void* ws,
                      size_t ws_bytes, void* stream);

/* Lebesgue constant: the largest value of the Lebesgue function Lambda
 * (see fh_lebesgue) on [x_0, x_{n-1}], the quantity the FH literature
 * reports per node family, n and d (Bos, De Marchi, Hormann and Klein,
 * Numer. Math. 2012).  Lambda = 1 at the nodes, so it is the largest of the
 * maxima over the n - 1 intervals [x_k, x_{k+1}]; each is searched for by a
 * grid zoom: `rounds` rounds, each sampling `samples` interior points
 * t_i = lo + (i + 1) h, h = (hi - lo) / (samples + 1), of the bracket
 * [lo, hi] (first the interval itself; the product and the sum rounded
 * separately), the next bracket being the two neighbours of the first
 * largest sample.  The search finds the maximum when Lambda has one local
 * maximum per interval; each round divides the bracket by (samples + 1)/2.
 *   nodes, n, d, w   as in fh_lebesgue (w may be NULL)
 *   samples          1..512 per round;  rounds 1..64
 *   lam_out          [n-1] per-interval maxima (the largest Lambda seen, first
 *                    seen on ties; NaN if no sample was a number), or NULL
 *   x_out            [n-1] where each was seen, or NULL
 *   best_out         [2] = {Lebesgue constant, its location}: the first
 *                    largest interval maximum (n = 1 gives {1, x_0}), or NULL
 *   prec             FH_FP64 (FH_FP32_SPLIT: FH_E_UNSUPPORTED; the zoom
 *                    compares values that differ in late digits)
 *   ws               fh_workspace_size(FH_OP_LEBESGUE_MAX, n, 0, d, prec)
 * All outputs are device arrays; at least one must be given.  Errors as in
 * fh_eval (node-order and weight-range problems set status bits). */
fh_status fh_lebesgue_max(const double* nodes, int64_t n, int32_t d, const double* w,
                          int32_t samples, int32_t rounds, double* lam_out, double* x_out,
                          double* best_out, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Several interpolants on the same nodes and points in one call: column c
 * (0 <= c < K) has degree d_host[c] and values values[c * n .. c * n + n - 1];
 * r_out[c * m + p] = r_c(x_p) and, if lambda_out is not NULL,
 * lambda_out[c * m + p] = Lambda_c(x_p).  The reciprocals 1 / (x_p - x_k)
 * are computed once for all columns (a sweep over d, or vector-valued data:
 * when all degrees are equal the weights, D and Lambda are shared too).
 * Every column's results are those of fh_eval (FH_FP64) bit for bit with
 * one point per lane, groups of eight and no node split (launch variant 3).
 *   K        1..64;  d_host: host array of K degrees, each in 0..n-1
 *   values   device [K][n];  r_out, lambda_out: device [K][m]
 *   ws       fh_multi_workspace_size(n, K) bytes (status block as in fh_eval)
 * Errors as in fh_eval (FH_E_DEGREE for a degree out of range). */
size_t fh_multi_workspace_size(int64_t n, int32_t K);
fh_status fh_eval_multi(const double* nodes, const double* values, int64_t n,
                        const int32_t* d_host, int32_t K, const double* x, int64_t m,
                        double* r_out, double* lambda_out, void* ws, size_t ws_bytes,
                        void* stream);

/* Derivative of the interpolant: r(x_p) (r_out, may be NULL) and r'(x_p)
 * (dr_out) at m points.  Away from the nodes r' = (r E - F) / D with
 * D = sum a_k, E = sum a_k / (x - x_k), F = sum a_k f_k / (x - x_k)
 * (a_k = w_k / (x - x_k)), the derivative of N / D; at an exact hit
 * x_p == x_j the node formula r'(x_j) = sum_{k!=j} (w_k/w_j)(f_k - f_j) /
 * (x_j - x_k) (Schneider & Werner 1986).  NaN and infinite points give NaN.
 * w, prec, ws (fh_workspace_size(FH_OP_EVAL, ...)) and the status block
 * behave as in fh_eval; FH_FP32_SPLIT runs the sums with binary32 terms as
 * the split evaluation does. */
fh_status fh_eval_deriv(const double* nodes, const double* values, int64_t n, int32_t d,
                        const double* x, int64_t m, double* r_out, double* dr_out,
                        const double* w, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of L = sum_p grad_r[p] * r(x_p) (any output may be NULL):
 *   grad_values [n]  dL/df_k    = sum_p g_p a_pk / D_p
 *   grad_x      [m]  dL/dx_p    = g_p sum_k a_pk (r_p - f_k) / ((x_p - x_k) D_p)
 *   grad_nodes  [n]  dL/dx_k    = sum_p g_p a_pk (f_k - r_p) / ((x_p - x_k) D_p)
 *                                 + sum_j dL/dw_j dw_j/dx_k   (total derivative)
 * At a hit x_p == x_j: dL/df_j gets g_p, dL/dx_p = g_p r'(x_j) with the node
 * formula r'(x_j) = sum_{k!=j} (w_k/w_j)(f_k - f_j)/(x_j - x_k) (Schneider &
 * Werner 1986), dL/dx_j gets -g_p r'(x_j), and the weights get nothing.
 * Per-node sums over points are reduced in a fixed order (deterministic).
 * prec = FH_FP32_SPLIT runs the pair terms in binary32 as fh_eval does (node
 * and point coordinates as binary32 head/tail pairs, weights and the point
 * factors g_p / D_p scaled by the same power of two, binary32 partial sums
 * over 32 terms added into binary64); data that leave the binary32 range
 * (node span outside [2^-20, 2^20], points more than one span outside the
 * nodes, g_p / D_p beyond 2^+-50 after scaling) take binary64 per-pair
 * paths, so the split gradients stay within about 2^-17 of the binary64
 * ones relative to the sums of their terms' magnitudes.
 *   ws  workspace of fh_workspace_size(FH_OP_BACKWARD, n, m, d, prec)      */
fh_status fh_eval_backward(const double* nodes, const double* values, int64_t n, int32_t d,
                           const double* x, int64_t m, const double* grad_r, double* grad_values,
                           double* grad_x, double* grad_nodes, int32_t prec, void* ws,
                           size_t ws_bytes, void* stream);

/* The adjoint in two steps that share their work, for callers that run a
 * forward evaluation and later its adjoint (automatic differentiation; the
 * saved-state form of the adjoint of L = sum_p grad_r[p] r(x_p)).
 *
 * fh_eval_forward: r(x_p) into r_out [m] and, in ws, the node table and what
 * the adjoint needs per point for unit loss weights: 1/D_p, r_p, and at an
 * exact hit x_p == x_j the flag and the node formula r'(x_j) (Schneider &
 * Werner 1986).  NaN and infinite points give r = NaN.  dr_out [m]
 * (nullable): also the derivative r'(x_p) there, as fh_eval_deriv computes
 * it (the same bits), for a caller that will want dL/dx_p.  Binary64 r has
 * the bits of fh_eval with launch variant 4 (and of fh_eval_deriv) with or
 * without dr_out; split r: fh_eval's split evaluation without dr_out,
 * fh_eval_deriv's with it.
 *
 * fh_eval_backward_saved: the gradients of fh_eval_backward (same
 * definitions, hit rules, outputs and NULL conventions) from that state and
 * the loss weights grad_r [m], without evaluating N_p and D_p again.  dr
 * (nullable): the forward's dr_out; with it dL/dx_p = grad_r[p] dr[p] and
 * the node gradients come from one pass over the (point, node) pairs with
 * the per-node sums S1..S4; without it, binary64, that same pass also forms
 * dL/dx_p, each reciprocal formed once for both: per point, the terms over
 * the lane's nodes, then across the wave (an LDS transpose) and over node
 * tile groups, all in a fixed order (deterministic).  The state is read, not
 * changed: the backward may run any number of times on one forward.
 *
 * Both take ws of fh_workspace_size(FH_OP_BACKWARD_SAVED, n, m, d, prec) and
 * must see the same nodes, n, d, x, m and prec; values are read by the
 * forward only.  Between the two calls the workspace must not be used by
 * another call.  prec = FH_FP32_SPLIT: with dr_out the forward runs the
 * split point pass for unit loss weights (r and r' with fh_eval_deriv's
 * bits) and keeps its binary64 and binary32 point records; the backward
 * scales them by grad_r and runs the split node pass alone.  Without dr_out
 * the forward is fh_eval's split evaluation and the backward the split
 * fh_eval_backward passes on the node table the forward packed.  Errors as in
 * fh_eval_backward; a backward on a workspace its forward did not fill
 * gives unspecified values. */
fh_status fh_eval_forward(const double* nodes, const double* values, int64_t n, int32_t d,
                          const double* x, int64_t m, double* r_out, double* dr_out,
                          int32_t prec, void* ws, size_t ws_bytes, void* stream);
fh_status fh_eval_backward_saved(const double* nodes, int64_t n, int32_t d, const double* x,
                                 int64_t m, const double* dr, const double* grad_r,
                                 double* grad_values, double* grad_x, double* grad_nodes,
                                 int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Batched evaluation of `count` independent interpolants of uneven sizes in
 * one captured HIP graph.  Instance i owns nodes/values
 * [node_off[i], node_off[i+1]) and points/outputs [pt_off[i], pt_off[i+1])
 * of the concatenated (CSR) device arrays, with node_off/pt_off the running
 * sums of n_host/m_host.
 *   fh_batch_create  validates the host arrays (n_i >= 1, 0 <= d_i <= n_i-1,
 *                    m_i >= 0), builds the longest-first work list, allocates
 *                    the batch's own device memory, and captures the weight
 *                    pass and the persistent evaluation kernel into a graph.
 *                    The device arrays are referenced, not copied: they must
 *                    stay allocated and in place until fh_batch_destroy.
 *   fh_eval_batched  launches the graph on `stream` (one hipGraphLaunch).
 *   fh_batch_destroy frees the batch (after its launches have completed). */
typedef struct fh_batch fh_batch;
fh_status fh_batch_create(fh_batch** out, int32_t count, const int64_t* n_host,
                          const int32_t* d_host, const int64_t* m_host, const double* nodes_cat,
                          const double* values_cat, const double* x_cat, double* r_cat,
                          double* lambda_cat, int32_t prec, void* stream);
fh_status fh_eval_batched(fh_batch* b, void* stream);
fh_status fh_batch_destroy(fh_batch* b);
/* Sticky device status bits of a batch (synchronizes the stream, clears). */
fh_status fh_batch_status(fh_batch* b, void* stream, uint32_t* bits_out);

/* Kernel-variant selection (the autotuner's interface).  Each evaluation
 * kernel exists in several launch variants: points per lane, node group size
 * of the shared reciprocal, node split across the waves of a block, the node
 * block of the Lebesgue sums, and (batches) the passes per work item.  The
 * variant for a call is looked up by (kernel family, ceil(log2 of n rounded
 * up to 64), ceil(log2 m)) in a per-process table; shapes with no entry use
 * a built-in table measured on MI355X, then a size rule.  Whether Lambda is
 * requested does not enter the choice, so r has the same bits with and
 * without it.  Kernel families: the precisions FH_FP64 and FH_FP32_SPLIT for
 * fh_eval / fh_lebesgue / fh_eval_prepared, and FH_TUNE_BATCHED_FP64 /
 * FH_TUNE_BATCHED_SPLIT for fh_batch_create (keyed by the mean n and the
 * total number of points; read when a batch is created).  All variants
 * compute the same quantities to the same error bound; they differ in speed
 * and, where their summation order differs, in the last bits.
 *   fh_variant_count / fh_variant_shape  enumerate the variants of a family
 *                  (points per lane, group size, node split);
 *   fh_variant_lebesgue_block  the node block length U of a variant whose
 *                  sums are taken by blocks (they use the alternating signs
 *                  of the weights: one multiply-add per pair serves both
 *                  sum_k a_k and sum_k |a_k|), 0 for plain sums, -1 for a bad
 *                  family or id.  Such a variant runs plain sums when caller
 *                  weights do not alternate strictly in sign (w_k w_{k+1} < 0
 *                  for every k; Floater-Hormann weights always do); r does not
 *                  depend on whether Lambda is requested.  Batched split
 *                  variants take tiles of 32, batched binary64 variants 16 or
 *                  plain sums;
 *   fh_variant_node_pairs  1 if a binary64 variant sums its node blocks
 *                  by pairs of records (k, k+2) -- one rational term per pair,
 *                  w_a/(x - x_a) + w_b/(x - x_b) = (B x'' + J)/(x''^2 - hh^2) --
 *                  with the blocks next to each point summed node by node
 *                  afterwards, 0 otherwise, -1 for a bad family or id;
 *   fh_variant_octets  1 if a binary64 variant also sums the node blocks
 *                  far from a point by octets (the eight even, and the eight
 *                  odd, records of a block as one rational function in
 *                  monomial form; a block serves the points at least two
 *                  whole blocks beyond the blocks of their neighbouring
 *                  nodes, and only tables whose every block passed the
 *                  octet error test use them), 0 otherwise, -1 for a bad
 *                  family or id.  Such a launch sorts the points by node
 *                  block first, which needs the workspace room that
 *                  fh_workspace_size(FH_OP_EVAL, n, m, ...) includes for m
 *                  points (n <= 65536, m < 2^31); with less room the call
 *                  runs the pair variant of the same shape (other bits),
 *                  as fh_eval_noalloc always does, and FH_LOG=1 reports it;
 *   fh_variant_strip_points  points one block covers (single-interpolant
 *                  families) or one work item (batched families), -1 for a
 *                  bad family or id;
 *   fh_tune_set    records variant `id` of family `prec` for the shape bucket
 *                  of (n, m) (id = -1 removes the entry);
 *   fh_tune_force  pins variant `id` of a family for every shape (-1
 *                  releases it);
 *   fh_tune_get    the variant a call with (n, m) would use now.
 * The table is process-wide and guarded by a mutex.  With the environment
 * variable FH_AUTOTUNE_CACHE naming a table saved by the autotuner
 * (paper_1606_06508_amd/autotune.py: JSON with "arch" and "entries"), the
 * library installs it on first use when its "arch" is the device's; FH_LOG=1
 * reports on stderr every new (shape, variant) choice, where it came from
 * (forced, tuned, built-in), and each batch's launch shape. */
enum { FH_TUNE_BATCHED_FP64 = 2, FH_TUNE_BATCHED_SPLIT = 3 };
int32_t fh_variant_count(int32_t prec);
fh_status fh_variant_shape(int32_t prec, int32_t id, int32_t* points_per_lane, int32_t* group,
                           int32_t* node_split);
int32_t fh_variant_lebesgue_block(int32_t prec, int32_t id);
int32_t fh_variant_node_pairs(int32_t prec, int32_t id);
int32_t fh_variant_octets(int32_t prec, int32_t id);
int64_t fh_variant_strip_points(int32_t prec, int32_t id);
fh_status fh_tune_set(int32_t prec, int64_t n, int64_t m, int32_t id);
fh_status fh_tune_force(int32_t prec, int32_t id);
int32_t fh_tune_get(int32_t prec, int64_t n, int64_t m);

/* The launch variant a batch runs (of family FH_TUNE_BATCHED_FP64 or
 * FH_TUNE_BATCHED_SPLIT, chosen when it was created) and the points of one
 * of its work items; -1 for NULL. */
int32_t fh_batch_variant(const fh_batch* b);
int64_t fh_batch_strip_points(const fh_batch* b);

/* Synchronizes `stream`, reads the workspace status word into *bits_out,
 * clears it, and returns the status of the most severe set bit, in the
 * order FH_E_NONFINITE, FH_E_NODES, FH_E_RANGE (FH_OK if no bit is set). */
fh_status fh_device_status(void* ws, void* stream, uint32_t* bits_out);

/* Static, human-readable name of a status code. */
const char* fh_status_string(int32_t s);

#ifdef __cplusplus
}
#endif
#endif /* FH_H */
