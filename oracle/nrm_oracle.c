/*
 * nrm_oracle.c -- plain scalar reference of the vector and quaternion
 * normalization of W. F. Mascarenhas, "Fast and accurate normalization of
 * vectors and quaternions": the length r = ||x|| and the direction x / r of
 * x in R^2, R^3 and R^4, computed by
 *   - the scaling algorithms (Scale2D / Scale3D of Section 2, Normalize2D /
 *     Normalize3D of Section 3, Normalize4D of Section 4) with the binary32
 *     and binary64 parameters of Table 2;
 *   - the quotient algorithms of the Introduction (Algorithm 1 for any
 *     dimension, Algorithm 2 for three dimensions);
 *   - the naive formula r = sqrt(sum x_k^2), h = 1/r, x_k h.
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers.  The product library
 * (HIP kernels behind the C ABI) shares no code, header, table or helper
 * with this file and never calls it.
 *
 * Every operation is one IEEE operation of the working precision, in the
 * order the algorithms state it: sums of squares left to right, one
 * correctly rounded square root, one division for h, products by h.  Built
 * with -ffp-contract=off (no fused multiply-add) and without fast-math, so a
 * machine that rounds every operation the same way gets the same bits.
 *
 * Readings where the printed algorithms are ambiguous or garbled:
 *   - the scaling procedures return the INVERSE of the scale factor
 *     (1, 1/sigma_max or 1/sigma_min) with the scaled vector, and the
 *     normalization procedures return that inverse times r~ (the printed
 *     return line multiplies by "r");
 *   - the largest magnitude m is found with the comparison tree of each
 *     procedure; the quaternion tree needs an "else" before its last
 *     assignment m <- |x_4| (as in Scale3D), otherwise a zero-free input
 *     with |x_1| >= |x_2|, |x_3|, |x_4| would lose its maximum;
 *   - a zero vector gives r = 0 and a zero direction in 2D and 3D; the zero
 *     quaternion gives r = 0 and the direction (0, 0, 1, 0) (the printed
 *     return tuple has one entry too few; its four entries are kept as the
 *     direction);
 *   - the parameters are those of Table 2 (tau_min = 2^-49 / 2^-482,
 *     sigma_min = 2^100 / 2^592, tau_max = 2^62 / 2^510,
 *     sigma_max = 2^-66 / 2^-514); the closed form (tau) of Section 2
 *     gives tau_min = 2^-50 / 2^-484 instead;
 *   - Algorithm 1 divides the scaled components x_k / m by
 *     s = sqrt(sum (x_k / m)^2) and returns r = m s (dividing them by r, as
 *     printed, would not give a unit vector);
 *   - Algorithm 2: the sign of the pivot is copysign(1, x_p);
 *   - the zero exits of Scale3D and Normalize4D are taken only when the
 *     entries that the tree compared with "<" alone are not NaN: as printed,
 *     (0, NaN, 0) would leave through the zero exit and lose its NaN, which
 *     contradicts the NaN statement of Section 2 (NaN in some input entry if
 *     and only if NaN in some output entry); with the check such a vector
 *     takes the sigma_min branch and every output is NaN.
 *
 * Build: gcc -O2 -std=c11 -fno-fast-math -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>

enum { NRO_OK = 0, NRO_E_ARG = 1 };
enum { NRO_SCALING = 0, NRO_QUOTIENT = 1, NRO_QUOTIENT_PIVOT = 2, NRO_NAIVE = 3 };

/* The parameters of Table 2. */
#define TMIN_F 0x1p-49f
#define SMIN_F 0x1p100f
#define TMAX_F 0x1p62f
#define SMAX_F 0x1p-66f
#define TMIN_D 0x1p-482
#define SMIN_D 0x1p592
#define TMAX_D 0x1p510
#define SMAX_D 0x1p-514

/*
 * One instantiation per working precision T.  SQRT, FABS and COPYSIGN are
 * the functions of T (SQRT correctly rounded), so no operation leaves T.
 */
#define NRO_DEFINE(T, SFX, SQRT, FABS, COPYSIGN, ONE, TMIN, SMIN, TMAX, SMAX)                               \
                                                                                            \
  /* Scale2D: returns the inverse scale s and the scaled vector y. */                       \
  static T scale2_##SFX(const T* x, T* y) {                                                 \
    T m = FABS(x[0]);                                                                       \
    if (m >= FABS(x[1])) {                                                                  \
      if (m == 0) {                                                                         \
        y[0] = y[1] = 0;                                                                    \
        return 0;                                                                           \
      }                                                                                     \
    } else {                                                                                \
      m = FABS(x[1]);                                                                       \
    }                                                                                       \
    if (m >= TMIN) {                                                                        \
      if (m <= TMAX) {                                                                      \
        y[0] = x[0];                                                                        \
        y[1] = x[1];                                                                        \
        return ONE;                                                                         \
      }                                                                                     \
      y[0] = SMAX * x[0];                                                                   \
      y[1] = SMAX * x[1];                                                                   \
      return ONE / SMAX;                                                                    \
    }                                                                                       \
    y[0] = SMIN * x[0];                                                                     \
    y[1] = SMIN * x[1];                                                                     \
    return ONE / SMIN;                                                                      \
  }                                                                                         \
                                                                                            \
  /* Scale3D. */                                                                            \
  static T scale3_##SFX(const T* x, T* y) {                                                 \
    T m = FABS(x[0]);                                                                       \
    if (m < FABS(x[1])) {                                                                   \
      m = FABS(x[1]);                                                                       \
      if (m < FABS(x[2])) m = FABS(x[2]);                                                   \
    } else {                                                                                \
      if (m >= FABS(x[2])) {                                                                \
        if (m == 0 && x[1] == x[1]) {                                                       \
          y[0] = y[1] = y[2] = 0;                                                           \
          return 0;                                                                         \
        }                                                                                   \
      } else {                                                                              \
        m = FABS(x[2]);                                                                     \
      }                                                                                     \
    }                                                                                       \
    if (m >= TMIN) {                                                                        \
      if (m <= TMAX) {                                                                      \
        for (int k = 0; k < 3; ++k) y[k] = x[k];                                            \
        return ONE;                                                                         \
      }                                                                                     \
      for (int k = 0; k < 3; ++k) y[k] = SMAX * x[k];                                       \
      return ONE / SMAX;                                                                    \
    }                                                                                       \
    for (int k = 0; k < 3; ++k) y[k] = SMIN * x[k];                                         \
    return ONE / SMIN;                                                                      \
  }                                                                                         \
                                                                                            \
  /* The scaling part of Normalize4D; returns 0 for the zero quaternion. */                 \
  static T scale4_##SFX(const T* x, T* y) {                                                 \
    T m = FABS(x[0]);                                                                       \
    if (m < FABS(x[1])) {                                                                   \
      m = FABS(x[1]);                                                                       \
      if (m < FABS(x[2])) m = FABS(x[2]);                                                   \
      if (m < FABS(x[3])) m = FABS(x[3]);                                                   \
    } else {                                                                                \
      if (m < FABS(x[2])) {                                                                 \
        m = FABS(x[2]);                                                                     \
        if (m < FABS(x[3])) m = FABS(x[3]);                                                 \
      } else {                                                                              \
        if (m >= FABS(x[3])) {                                                              \
          if (m == 0 && x[1] == x[1] && x[2] == x[2]) {                                     \
            y[0] = y[1] = y[2] = y[3] = 0;                                                  \
            return 0;                                                                       \
          }                                                                                 \
        } else {                                                                            \
          m = FABS(x[3]);                                                                   \
        }                                                                                   \
      }                                                                                     \
    }                                                                                       \
    if (m >= TMIN) {                                                                        \
      if (m <= TMAX) {                                                                      \
        for (int k = 0; k < 4; ++k) y[k] = x[k];                                            \
        return ONE;                                                                         \
      }                                                                                     \
      for (int k = 0; k < 4; ++k) y[k] = SMAX * x[k];                                       \
      return ONE / SMAX;                                                                    \
    }                                                                                       \
    for (int k = 0; k < 4; ++k) y[k] = SMIN * x[k];                                         \
    return ONE / SMIN;                                                                      \
  }                                                                                         \
                                                                                            \
  /* Normalize2D / Normalize3D / Normalize4D. */                                            \
  static void scaling_##SFX(int dim, const T* x, T* r, T* xh) {                             \
    T y[4];                                                                                 \
    const T s = dim == 2 ? scale2_##SFX(x, y)                                               \
                         : (dim == 3 ? scale3_##SFX(x, y) : scale4_##SFX(x, y));            \
    if (s == 0) {                                                                           \
      *r = 0;                                                                               \
      for (int k = 0; k < dim; ++k) xh[k] = 0;                                              \
      if (dim == 4) xh[2] = ONE;                                                            \
      return;                                                                               \
    }                                                                                       \
    T acc = y[0] * y[0];                                                                    \
    for (int k = 1; k < dim; ++k) acc = acc + y[k] * y[k];                                  \
    const T rt = SQRT(acc);                                                                 \
    const T h = ONE / rt;                                                                   \
    *r = s * rt;                                                                            \
    for (int k = 0; k < dim; ++k) xh[k] = h * y[k];                                         \
  }                                                                                         \
                                                                                            \
  /* Algorithm 1 (any dimension). */                                                        \
  static void quotient_##SFX(int dim, const T* x, T* r, T* xh) {                            \
    T m = FABS(x[0]);                                                                       \
    for (int k = 1; k < dim; ++k)                                                           \
      if (FABS(x[k]) > m) m = FABS(x[k]);                                                   \
    if (m == 0) {                                                                           \
      *r = 0;                                                                               \
      for (int k = 0; k < dim; ++k) xh[k] = x[k];                                           \
      return;                                                                               \
    }                                                                                       \
    T y[4];                                                                                 \
    for (int k = 0; k < dim; ++k) y[k] = x[k] / m;                                          \
    T acc = y[0] * y[0];                                                                    \
    for (int k = 1; k < dim; ++k) acc = acc + y[k] * y[k];                                  \
    const T sq = SQRT(acc);                                                                 \
    *r = m * sq;                                                                            \
    for (int k = 0; k < dim; ++k) xh[k] = y[k] / sq;                                        \
  }                                                                                         \
                                                                                            \
  /* Algorithm 2 (three dimensions): pivot p, the other two in order. */                    \
  static void quotient_pivot_##SFX(const T* x, T* r, T* xh) {                               \
    int p;                                                                                  \
    if (FABS(x[0]) > FABS(x[1])) {                                                          \
      p = FABS(x[2]) > FABS(x[0]) ? 2 : 0;                                                  \
    } else {                                                                                \
      if (FABS(x[2]) >= FABS(x[1])) {                                                       \
        if (x[2] == 0) {                                                                    \
          *r = 0;                                                                           \
          xh[0] = xh[1] = xh[2] = 0;                                                        \
          return;                                                                           \
        }                                                                                   \
        p = 2;                                                                              \
      } else {                                                                              \
        p = 1;                                                                              \
      }                                                                                     \
    }                                                                                       \
    const int a = p == 0 ? 1 : 0, b = p == 2 ? 1 : 2;                                       \
    const T qa = x[a] / x[p], qb = x[b] / x[p];                                             \
    const T h = SQRT(ONE + qa * qa + qb * qb);                                              \
    *r = FABS(x[p]) * h;                                                                    \
    const T xp = COPYSIGN(ONE, x[p]) / h;                                                   \
    xh[a] = qa * xp;                                                                        \
    xh[b] = qb * xp;                                                                        \
    xh[p] = xp;                                                                             \
  }                                                                                         \
                                                                                            \
  static void naive_##SFX(int dim, const T* x, T* r, T* xh) {                               \
    T acc = x[0] * x[0];                                                                    \
    for (int k = 1; k < dim; ++k) acc = acc + x[k] * x[k];                                  \
    const T rt = SQRT(acc);                                                                 \
    const T h = ONE / rt;                                                                   \
    *r = rt;                                                                                \
    for (int k = 0; k < dim; ++k) xh[k] = h * x[k];                                         \
  }                                                                                         \
                                                                                            \
  /* x: n vectors of dim entries (row major); r[n] and xh[n][dim] may be    */              \
  /* NULL.                                                                  */              \
  int nro_normalize_##SFX(int dim, int method, const T* x, int64_t n, T* r, T* xh) {        \
    if (dim < 2 || dim > 4 || n < 0 || (n > 0 && x == 0)) return NRO_E_ARG;                 \
    if (method < NRO_SCALING || method > NRO_NAIVE) return NRO_E_ARG;                       \
    if (method == NRO_QUOTIENT_PIVOT && dim != 3) return NRO_E_ARG;                         \
    for (int64_t i = 0; i < n; ++i) {                                                       \
      T rr, hh[4];                                                                          \
      const T* v = x + i * dim;                                                             \
      if (method == NRO_SCALING)                                                            \
        scaling_##SFX(dim, v, &rr, hh);                                                     \
      else if (method == NRO_QUOTIENT)                                                      \
        quotient_##SFX(dim, v, &rr, hh);                                                    \
      else if (method == NRO_QUOTIENT_PIVOT)                                                \
        quotient_pivot_##SFX(v, &rr, hh);                                                   \
      else                                                                                  \
        naive_##SFX(dim, v, &rr, hh);                                                       \
      if (r) r[i] = rr;                                                                     \
      if (xh)                                                                               \
        for (int k = 0; k < dim; ++k) xh[i * dim + k] = hh[k];                              \
    }                                                                                       \
    return NRO_OK;                                                                          \
  }

NRO_DEFINE(float, f32, sqrtf, fabsf, copysignf, 1.0f, TMIN_F, SMIN_F, TMAX_F, SMAX_F)
NRO_DEFINE(double, f64, sqrt, fabs, copysign, 1.0, TMIN_D, SMIN_D, TMAX_D, SMAX_D)

/* The parameters, for the tests that check them against Table 2's
   conditions: {tau_min, sigma_min, tau_max, sigma_max}. */
void nro_params_f32(float* p) {
  p[0] = TMIN_F;
  p[1] = SMIN_F;
  p[2] = TMAX_F;
  p[3] = SMAX_F;
}
void nro_params_f64(double* p) {
  p[0] = TMIN_D;
  p[1] = SMIN_D;
  p[2] = TMAX_D;
  p[3] = SMAX_D;
}
