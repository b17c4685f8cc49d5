/* nrm.h -- batched vector and quaternion normalization on MI355X (gfx950).
 *
 * The length r = ||x|| and the direction x / r of n vectors in R^2, R^3 or
 * R^4 (quaternions), following W. F. Mascarenhas, "Fast and accurate
 * normalization of vectors and quaternions":
 *   NRM_SCALING         the scaling algorithms: Scale2D / Scale3D (Section 2)
 *                       with Normalize2D / Normalize3D (Section 3) and
 *                       Normalize4D (Section 4), parameters of Table 2;
 *                       Lemma 1 (R^2, R^3) and Lemma 2 (quaternions) bound
 *                       their errors;
 *   NRM_QUOTIENT        Algorithm 1 of the Introduction (divide by the
 *                       largest magnitude), any dimension;
 *   NRM_QUOTIENT_PIVOT  Algorithm 2 of the Introduction (divide by the
 *                       largest entry), three dimensions only;
 *   NRM_NAIVE           r = sqrt(sum x_k^2), h = 1/r, x_k h.
 * Every step is one IEEE operation of the working precision in the order
 * the algorithms state (sums of squares left to right, no fused
 * multiply-add, correctly rounded square root and division), so the
 * results are reproducible bit for bit.
 *
 * Conventions (where the printed algorithms are ambiguous):
 *   - a zero vector gives r = 0 and the zero direction; the zero quaternion
 *     gives r = 0 and the direction (0, 0, 1, 0);
 *   - NaN in some input entry gives NaN in r and in every direction entry
 *     (scaling method): the zero exits of the comparison trees are not
 *     taken when an entry compared only with "<" is NaN;
 *   - finite input gives a finite direction (r itself overflows only when
 *     ||x|| exceeds the largest finite value);
 *   - Algorithm 1 returns r = m s with s = sqrt(sum (x_k/m)^2) and the
 *     direction (x_k/m)/s.
 *
 * Arguments (all pointers are device pointers owned by the caller; calls
 * are asynchronous on `stream`, a hipStream_t passed as void*, NULL = the
 * null stream):
 *   x         input vectors; layout NRM_AOS: x[n][dim] (entries of one vector
 *             adjacent), NRM_SOA: x[dim][n] (entry k of vector i at k n + i);
 *   n         number of vectors (>= 0; 0 launches nothing);
 *   r_out     [n] lengths, or NULL;
 *   xhat_out  directions in the layout of x, or NULL (not both NULL when
 *             n > 0); may not overlap x;
 *   layout    nrm_layout; method  nrm_method.
 * Returns FH_OK, FH_E_ARG (n < 0, a NULL array that is needed, an unknown
 * layout or method, NRM_QUOTIENT_PIVOT outside three dimensions) before any
 * launch, or FH_E_HIP if the launch fails. */
#ifndef NRM_H
#define NRM_H

#include <stdint.h>

#include "fh.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { NRM_SCALING = 0, NRM_QUOTIENT = 1, NRM_QUOTIENT_PIVOT = 2, NRM_NAIVE = 3 } nrm_method;
typedef enum { NRM_AOS = 0, NRM_SOA = 1 } nrm_layout;

fh_status nrm_normalize2_f32(const float* x, int64_t n, float* r_out, float* xhat_out,
                             int32_t layout, int32_t method, void* stream);
fh_status nrm_normalize3_f32(const float* x, int64_t n, float* r_out, float* xhat_out,
                             int32_t layout, int32_t method, void* stream);
fh_status nrm_normalize4_f32(const float* x, int64_t n, float* r_out, float* xhat_out,
                             int32_t layout, int32_t method, void* stream);
fh_status nrm_normalize2_f64(const double* x, int64_t n, double* r_out, double* xhat_out,
                             int32_t layout, int32_t method, void* stream);
fh_status nrm_normalize3_f64(const double* x, int64_t n, double* r_out, double* xhat_out,
                             int32_t layout, int32_t method, void* stream);
fh_status nrm_normalize4_f64(const double* x, int64_t n, double* r_out, double* xhat_out,
                             int32_t layout, int32_t method, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NRM_H */
