/*
 * rcholqr_oracle.c -- plain, slow, FP64 CPU oracle for randomized Cholesky QR.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * (the HIP library under paper_2210_09953_amd/) never links, calls or
 * includes anything from here, and this file shares no code with it: the
 * Philox generator, the Gaussian transform, the Householder QR, the
 * substitutions and the Cholesky factorisation below are written
 * independently from their published definitions.
 *
 * What it computes (Balabanov, "Randomized Cholesky QR factorizations"):
 *   Algorithm 2 (RCholeskyQR):  P = Theta X;  [S, R] = QR(P);  Q = X R^{-1}
 *   Algorithm 3 (RCholeskyQR2): Algorithm 2, then A = Q^T Q; R' = chol(A);
 *                               R = R' R;  Q = Q R'^{-1}
 * with Theta a k x m oblivious subspace embedding applied as a function
 * handle driven by a seeded counter-based generator (Section 2, "seeded
 * random number generator, implying negligible memory").  The step-2 QR is
 * Householder, the choice made in the numerical experiments (Section 6.1);
 * step 3 is row-wise forward substitution (Section 3.1 cost discussion and
 * the Higham Thm 8.5 argument of Section 5.1).
 *
 * Readings of points the paper leaves open (all listed in the design doc):
 *   - R has a positive diagonal (sign fix after Householder), so that the
 *     2-pass (Q, R) is the unique thin QR and can be compared with LAPACK.
 *   - chol() is the upper factor with A = R'^T R'; the R update multiplies
 *     on the left, R <- R' R_s.
 *   - Gaussian Theta has entries z / sqrt(k); the 1/sqrt(k) is applied to
 *     the accumulated sketch.  Rademacher: +-1 / sqrt(k).  CountSketch: one
 *     +-1 per column at a hashed row, no scaling.
 *   - Theta's entries come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     SC'11), key = seed, then the transforms below.  Gaussian: counter =
 *     (row j of X, pair of Theta rows, stream tag).  Rademacher: counter =
 *     (block j >> 7 of 128 rows of X, Theta row, stream tag), one bit per
 *     row of X.  CountSketch: counter = (row j of X, 0, stream tag).
 *
 * All arithmetic is IEEE binary64, round-to-nearest; compile with
 * -ffp-contract=off so that no multiply-add is fused behind our back (the
 * Gaussian transform uses explicit fma() where it wants one).
 *
 * Pins (tests/test_oracle_pins.py): Philox against an independent library
 * implementation; transforms against mpmath; distributions against exact
 * laws (KS, moments); sketch against a materialised Theta times X; QR,
 * substitution and Cholesky against LAPACK; closed forms (n = 1, identity
 * sketch, orthonormal input); Theorem 5.2 invariants; adjoint against
 * finite differences and against autograd of LAPACK's QR.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_GAUSSIAN 0
#define ORC_RADEMACHER 1
#define ORC_COUNTSKETCH 2
#define ORC_IDENTITY 99

/* Stream tags occupying the fourth counter word (one stream per use). */
#define ORC_TAG_GAUSS 0x47415553u  /* "GAUS" */
#define ORC_TAG_RADEM 0x52414445u  /* "RADE" */
#define ORC_TAG_COUNT 0x434F554Eu  /* "COUN" */

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon et al. SC'11: each round multiplies words 0 */
/* and 2 by the two round multipliers, and recombines high halves with    */
/* words 1, 3 and the round key; the key is bumped by the two Weyl        */
/* constants (golden ratio, sqrt(3)-1) between rounds.                    */
/* ------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL_A;
      k1 += PHILOX_WEYL_B;
    }
    uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
    uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
    uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
    uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
    uint32_t n0 = hi_b ^ c1 ^ k0;
    uint32_t n1 = lo_b;
    uint32_t n2 = hi_a ^ c3 ^ k1;
    uint32_t n3 = lo_a;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_at(uint64_t seed, int64_t j, uint32_t word2, uint32_t tag,
                      uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)((uint64_t)j & 0xffffffffu),
                     (uint32_t)((uint64_t)j >> 32), word2, tag};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* ------------------------------------------------------------------ */
/* Gaussian transform (Box & Muller 1958) with project-defined ln and    */
/* sin/cos of 2*pi*u built only from +, -, *, /, sqrt and fma, so that   */
/* any IEEE machine evaluating the same steps gets the same bits.        */
/* ------------------------------------------------------------------ */

/* ln(x) for finite x > 0:  x = f 2^e with f in [sqrt(2)/2, sqrt(2)),
 * s = (f-1)/(f+1),  ln f = 2 atanh(s) = 2 s sum_{i>=0} s^{2i}/(2i+1)
 * truncated after i = 12 (|s| <= 0.1716, the tail is below 2^-60),
 * ln x = e ln2_hi + (e ln2_lo + ln f) with ln 2 split so e*ln2_hi is exact. */
double orc_ln(double x) {
  uint64_t bits;
  memcpy(&bits, &x, 8);
  int e = (int)((bits >> 52) & 0x7ff);
  if (e == 0) { /* subnormal: scale into the normal range first */
    x = x * 0x1p54;
    memcpy(&bits, &x, 8);
    e = (int)((bits >> 52) & 0x7ff) - 54;
  }
  e -= 1023;
  uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
  double f;
  memcpy(&f, &mbits, 8); /* f in [1, 2) */
  if (f >= 0x1.6a09e667f3bcdp+0) { /* f >= sqrt(2): halve, exactly */
    f = f * 0.5;
    e += 1;
  }
  double s = (f - 1.0) / (f + 1.0);
  double s2 = s * s;
  static const double c[13] = {
      0x1.0000000000000p+0, 0x1.5555555555555p-2, 0x1.999999999999ap-3,
      0x1.2492492492492p-3, 0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4,
      0x1.3b13b13b13b14p-4, 0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5,
      0x1.af286bca1af28p-5, 0x1.8618618618618p-5, 0x1.642c8590b2164p-5,
      0x1.47ae147ae147bp-5};
  double p = c[12];
  for (int i = 11; i >= 0; --i) p = fma(p, s2, c[i]);
  double t = s * p;
  double lnf = t + t;
  double de = (double)e;
  const double LN2_HI = 0x1.62e42fee00000p-1;
  const double LN2_LO = 0x1.a39ef35793c76p-33;
  return de * LN2_HI + (de * LN2_LO + lnf);
}

/* sin and cos of 2*pi*u for u = b * 2^-53 with integer b in [0, 2^53).
 * Quadrant reduction is exact on the integer b: q = round(4u),
 * r = 4u - q in [-1/2, 1/2), x = r * pi/2 in [-pi/4, pi/4]; then Taylor
 * series of sin (through x^19) and cos (through x^20), and the quadrant
 * rotation. */
void orc_sincos2pi_dyadic(uint64_t b, double* s_out, double* c_out) {
  uint64_t q = (b + (1ull << 50)) >> 51; /* 0..4 */
  int64_t ri = (int64_t)b - (int64_t)(q << 51);
  double r = (double)ri * 0x1p-51;
  double x = r * 0x1.921fb54442d18p+0;
  double x2 = x * x;
  static const double S[9] = {
      -0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
      0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26, 0x1.6124613a86d09p-33,
      -0x1.ae7f3e733b81fp-41, 0x1.952c77030ad4ap-49, -0x1.2f49b46814157p-57};
  static const double C[9] = {
      0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-16,
      -0x1.27e4fb7789f5cp-22, 0x1.1eed8eff8d898p-29, -0x1.93974a8c07c9dp-37,
      0x1.ae7f3e733b81fp-45, -0x1.6827863b97d97p-53, 0x1.e542ba4020225p-62};
  double ps = S[8];
  for (int i = 7; i >= 0; --i) ps = fma(ps, x2, S[i]);
  double sn = fma(x * x2, ps, x);
  double pc = C[8];
  for (int i = 7; i >= 0; --i) pc = fma(pc, x2, C[i]);
  double cs = fma(x2 * x2, pc, fma(-0.5, x2, 1.0));
  switch ((int)(q & 3)) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
  }
}

/* Gaussian pair for Theta column j (= row j of X), Theta rows 2b and 2b+1. */
static void gauss_pair(uint64_t seed, int64_t j, uint32_t b, double* z0,
                       double* z1) {
  uint32_t w[4];
  philox_at(seed, j, b, ORC_TAG_GAUSS, w);
  uint64_t a = ((((uint64_t)w[0]) << 32) | w[1]) >> 11;
  uint64_t bb = ((((uint64_t)w[2]) << 32) | w[3]) >> 11;
  double u1 = (double)(a + 1) * 0x1p-53; /* (0, 1] */
  double rho = sqrt(-2.0 * orc_ln(u1));
  double sn, cs;
  orc_sincos2pi_dyadic(bb, &sn, &cs);
  *z0 = rho * cs;
  *z1 = rho * sn;
}

/* Rademacher sign for column offset r (0..127) of a 128-column block, from
 * the four Philox words of that block and Theta row: writing
 * r = 32 q + 4 t + e (q < 4, t < 8, e < 4), the sign is -1 when bit
 * 8 e + t of word q is set. */
static double radem_sign(const uint32_t w[4], int r) {
  int q = r >> 5, t = (r & 31) >> 2, e = r & 3;
  return ((w[q] >> (8 * e + t)) & 1u) ? -1.0 : 1.0;
}

/* Raw (unscaled) Theta entry at row i, column j. */
static double theta_raw(int kind, int64_t k, uint64_t seed, int64_t i,
                        int64_t j) {
  if (kind == ORC_GAUSSIAN) {
    double z0, z1;
    gauss_pair(seed, j, (uint32_t)(i >> 1), &z0, &z1);
    return (i & 1) ? z1 : z0;
  } else if (kind == ORC_RADEMACHER) {
    uint32_t w[4];
    philox_at(seed, j >> 7, (uint32_t)i, ORC_TAG_RADEM, w);
    return radem_sign(w, (int)(j & 127));
  } else if (kind == ORC_COUNTSKETCH) {
    uint32_t w[4];
    philox_at(seed, j, 0u, ORC_TAG_COUNT, w);
    int64_t h = (int64_t)(((uint64_t)w[0] * (uint64_t)k) >> 32);
    double s = (w[1] & 1u) ? -1.0 : 1.0;
    return (h == i) ? s : 0.0;
  } else { /* identity (test-only): k == m */
    return (i == j) ? 1.0 : 0.0;
  }
}

/* Materialise raw Theta(i0:i0+ni, j0:j0+nj) column-major into out (ld = ni). */
void orc_theta_block(int kind, int64_t k, int64_t m, uint64_t seed, int64_t i0,
                     int64_t ni, int64_t j0, int64_t nj, double* out) {
  (void)m;
  for (int64_t jj = 0; jj < nj; ++jj)
    for (int64_t ii = 0; ii < ni; ++ii)
      out[ii + jj * ni] = theta_raw(kind, k, seed, i0 + ii, j0 + jj);
}

/* CountSketch hash and sign of column j (exported for tests). */
void orc_countsketch_hash(int64_t k, uint64_t seed, int64_t j, int64_t* h,
                          double* s) {
  uint32_t w[4];
  philox_at(seed, j, 0u, ORC_TAG_COUNT, w);
  *h = (int64_t)(((uint64_t)w[0] * (uint64_t)k) >> 32);
  *s = (w[1] & 1u) ? -1.0 : 1.0;
}

/* Scaling applied to the accumulated sketch: 1/sqrt(k) for the dense
 * embeddings (Section 2, rescaled Gaussian), 1 otherwise. */
double orc_sketch_scale(int kind, int64_t k) {
  if (kind == ORC_GAUSSIAN || kind == ORC_RADEMACHER)
    return 1.0 / sqrt((double)k);
  return 1.0;
}

/* Algorithm 2 step 1: P = Theta X (k x n, ld = ldp).  Each Theta row i
 * is accumulated over j = 0..m-1 in order; Theta rows are independent so
 * they are shared out over threads without changing any sum. */
void orc_sketch(int kind, int64_t m, int64_t n, int64_t k, uint64_t seed,
                const double* X, int64_t ldx, double* P, int64_t ldp) {
  double scale = orc_sketch_scale(kind, k);
  if (kind == ORC_COUNTSKETCH) {
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < k; ++i) P[i + c * ldp] = 0.0;
    for (int64_t j = 0; j < m; ++j) {
      int64_t h;
      double s;
      orc_countsketch_hash(k, seed, j, &h, &s);
      for (int64_t c = 0; c < n; ++c) P[h + c * ldp] += s * X[j + c * ldx];
    }
    return;
  }
  if (kind == ORC_IDENTITY) {
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < k; ++i) P[i + c * ldp] = X[i + c * ldx];
    return;
  }
  /* Dense kinds, in groups of Theta rows: Gaussian pairs; Rademacher rows
 * one at a time (a row's draws cover 128 columns each). */
  int64_t rows_per_draw = (kind == ORC_GAUSSIAN) ? 2 : 1;
  int64_t ndraw = (k + rows_per_draw - 1) / rows_per_draw;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t d = 0; d < ndraw; ++d) {
    int64_t i0 = d * rows_per_draw;
    int64_t ni = (i0 + rows_per_draw <= k) ? rows_per_draw : (k - i0);
    double* acc = (double*)calloc((size_t)(ni * n), sizeof(double));
    double th[2];
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int64_t j = 0; j < m; ++j) {
      if (kind == ORC_GAUSSIAN) {
        double z0, z1;
        gauss_pair(seed, j, (uint32_t)(i0 >> 1), &z0, &z1);
        th[0] = z0;
        th[1] = z1; /* dropped when k is odd and this is the last pair */
      } else {
        if ((j & 127) == 0)
          philox_at(seed, j >> 7, (uint32_t)i0, ORC_TAG_RADEM, w);
        th[0] = radem_sign(w, (int)(j & 127));
      }
      for (int64_t c = 0; c < n; ++c) {
        double x = X[j + c * ldx];
        for (int64_t ii = 0; ii < ni; ++ii) acc[ii + c * ni] += th[ii] * x;
      }
    }
    for (int64_t c = 0; c < n; ++c)
      for (int64_t ii = 0; ii < ni; ++ii)
        P[i0 + ii + c * ldp] = scale * acc[ii + c * ni];
    free(acc);
  }
}

/* Algorithm 2 step 2: textbook Householder QR of P (k x n, k >= n), then a
 * sign fix D = sign(diag R) (sign(0) = +1) so that R_s = D R has a
 * positive diagonal and S = Q_hh D.  R (n x n, ld = ldr) gets the upper
 * triangle and zeros below; S (k x n, ld = lds) may be NULL.
 * Returns 0, or 1 if a diagonal entry of R_s is zero or not finite. */
int orc_householder_qr(int64_t k, int64_t n, const double* P, int64_t ldp,
                       double* R, int64_t ldr, double* S, int64_t lds) {
  double* A = (double*)malloc((size_t)(k * n) * sizeof(double));
  double* V = (double*)calloc((size_t)(k * n), sizeof(double));
  double* beta = (double*)calloc((size_t)n, sizeof(double));
  /* Each column enters scaled by 2^-e_c (e_c: the exponent of its largest
   * magnitude; 0 for a zero or non-finite column), as LAPACK's reflector
   * generation guards its norm, so that the sums of squares below cannot
   * underflow or overflow.  Householder QR commutes with a power-of-two
   * column scaling (QR(P D) = Q (R D)) without changing any rounding in the
   * normal range; R's columns are scaled back at the end. */
  int* cexp = (int*)calloc((size_t)n, sizeof(int));
  for (int64_t c = 0; c < n; ++c) {
    double mx = 0.0;
    int finite = 1;
    for (int64_t i = 0; i < k; ++i) {
      double a = fabs(P[i + c * ldp]);
      if (!isfinite(a)) finite = 0;
      else if (a > mx) mx = a;
    }
    if (finite && mx > 0.0) {
      int ex = 0;
      (void)frexp(mx, &ex);
      cexp[c] = ex - 1;
    }
    for (int64_t i = 0; i < k; ++i) A[i + c * k] = ldexp(P[i + c * ldp], -cexp[c]);
  }
  for (int64_t j = 0; j < n; ++j) {
    double nrm2 = 0.0;
    for (int64_t i = j; i < k; ++i) nrm2 += A[i + j * k] * A[i + j * k];
    double nrm = sqrt(nrm2);
    double x0 = A[j + j * k];
    double alpha = (x0 >= 0.0) ? -nrm : nrm; /* reflect away from x0 */
    double vtv = 0.0;
    V[j + j * k] = x0 - alpha;
    for (int64_t i = j + 1; i < k; ++i) V[i + j * k] = A[i + j * k];
    for (int64_t i = j; i < k; ++i) vtv += V[i + j * k] * V[i + j * k];
    beta[j] = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    /* A(j:k, j:n) <- (I - beta v v^T) A(j:k, j:n) */
    for (int64_t c = j; c < n; ++c) {
      double dot = 0.0;
      for (int64_t i = j; i < k; ++i) dot += V[i + j * k] * A[i + c * k];
      double f = beta[j] * dot;
      for (int64_t i = j; i < k; ++i) A[i + c * k] -= f * V[i + j * k];
    }
  }
  int status = 0;
  double* d = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t j = 0; j < n; ++j) {
    double rjj = A[j + j * k];
    d[j] = (rjj < 0.0) ? -1.0 : 1.0;
  }
  for (int64_t c = 0; c < n; ++c)
    for (int64_t r = 0; r < n; ++r)
      R[r + c * ldr] = (r <= c) ? ldexp(d[r] * A[r + c * k], cexp[c]) : 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double rjj = R[j + j * ldr];
    if (!(rjj > 0.0) || !isfinite(rjj)) status = 1;
  }
  if (S) {
    /* S = H_0 H_1 ... H_{n-1} [I_n; 0], accumulated from the last reflector. */
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < k; ++i) S[i + c * lds] = (i == c) ? 1.0 : 0.0;
    for (int64_t j = n - 1; j >= 0; --j) {
      for (int64_t c = 0; c < n; ++c) {
        double dot = 0.0;
        for (int64_t i = j; i < k; ++i) dot += V[i + j * k] * S[i + c * lds];
        double f = beta[j] * dot;
        for (int64_t i = j; i < k; ++i) S[i + c * lds] -= f * V[i + j * k];
      }
    }
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < k; ++i) S[i + c * lds] *= d[c];
  }
  free(cexp);
  free(d);
  free(beta);
  free(V);
  free(A);
  return status;
}

/* Algorithm 2 step 3: Q = X R^{-1} by forward substitution on each row
 * (q R = x, q_j = (x_j - sum_{l<j} q_l R_lj) / R_jj, l ascending). */
void orc_trsm_rows(int64_t m, int64_t n, const double* X, int64_t ldx,
                   const double* R, int64_t ldr, double* Q, int64_t ldq) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      double s = X[i + j * ldx];
      for (int64_t l = 0; l < j; ++l) s -= Q[i + l * ldq] * R[l + j * ldr];
      Q[i + j * ldq] = s / R[j + j * ldr];
    }
  }
}

/* Algorithm 3 step 2: A = Q^T Q (n x n, full symmetric), rows summed in order. */
void orc_gram(int64_t m, int64_t n, const double* Q, int64_t ldq, double* G,
              int64_t ldg) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < n; ++b) {
    for (int64_t a = 0; a <= b; ++a) {
      double s = 0.0;
      for (int64_t i = 0; i < m; ++i) s += Q[i + a * ldq] * Q[i + b * ldq];
      G[a + b * ldg] = s;
      G[b + a * ldg] = s;
    }
  }
}

/* Algorithm 3 step 3: upper Cholesky A = R'^T R' (MATLAB's chol).  Writes
 * the upper triangle of Rp and zeros below.  Returns 0, or 1000 + j
 * (0-based column) at the first non-positive or non-finite pivot. */
int orc_cholesky_upper(int64_t n, const double* G, int64_t ldg, double* Rp,
                       int64_t ldr) {
  for (int64_t c = 0; c < n; ++c)
    for (int64_t r = 0; r < n; ++r) Rp[r + c * ldr] = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double d = G[j + j * ldg];
    for (int64_t l = 0; l < j; ++l) d -= Rp[l + j * ldr] * Rp[l + j * ldr];
    if (!(d > 0.0) || !isfinite(d)) return (int)(1000 + j);
    double rjj = sqrt(d);
    Rp[j + j * ldr] = rjj;
    for (int64_t c = j + 1; c < n; ++c) {
      double s = G[j + c * ldg];
      for (int64_t l = 0; l < j; ++l) s -= Rp[l + j * ldr] * Rp[l + c * ldr];
      Rp[j + c * ldr] = s / rjj;
    }
  }
  return 0;
}

/* C = A B for upper triangular n x n A and B (the R <- R' R update). */
void orc_triu_product(int64_t n, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc) {
  for (int64_t c = 0; c < n; ++c)
    for (int64_t r = 0; r < n; ++r) {
      double s = 0.0;
      if (r <= c)
        for (int64_t l = r; l <= c; ++l) s += A[r + l * lda] * B[l + c * ldb];
      C[r + c * ldc] = s;
    }
}

/* Full Algorithm 2 (passes = 1) or Algorithm 3 (passes = 2).
 * Outputs: Q (m x n), R (n x n); optional S (k x n, Algorithm 2's
 * orthonormal sketch), Rs (sketch R), Rp (Cholesky factor, passes = 2).
 * Returns 0, 1 (sketch R rank failure), 2 (non-finite input) or 1000 + j
 * (Cholesky breakdown at column j). */
int orc_rcholqr(int kind, int passes, int64_t m, int64_t n, int64_t k,
                uint64_t seed, const double* X, int64_t ldx, double* Q,
                int64_t ldq, double* R, int64_t ldr, double* S, int64_t lds,
                double* Rs_out, double* Rp_out) {
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < m; ++i)
      if (!isfinite(X[i + c * ldx])) return 2;
  double* P = (double*)malloc((size_t)(k * n) * sizeof(double));
  double* Rs = (double*)malloc((size_t)(n * n) * sizeof(double));
  orc_sketch(kind, m, n, k, seed, X, ldx, P, k);
  int st = orc_householder_qr(k, n, P, k, Rs, n, S, lds);
  free(P);
  if (st != 0) {
    free(Rs);
    return st;
  }
  orc_trsm_rows(m, n, X, ldx, Rs, n, Q, ldq);
  if (Rs_out) memcpy(Rs_out, Rs, (size_t)(n * n) * sizeof(double));
  if (passes == 1) {
    for (int64_t c = 0; c < n; ++c)
      for (int64_t r = 0; r < n; ++r) R[r + c * ldr] = Rs[r + c * n];
    free(Rs);
    return 0;
  }
  double* G = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* Rp = (double*)malloc((size_t)(n * n) * sizeof(double));
  orc_gram(m, n, Q, ldq, G, n);
  st = orc_cholesky_upper(n, G, n, Rp, n);
  if (st == 0) {
    orc_triu_product(n, Rp, n, Rs, n, R, ldr);
    /* Q <- Q R'^{-1}, row by row (each row's solve reads only that row). */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
      for (int64_t j = 0; j < n; ++j) {
        double s = Q[i + j * ldq];
        for (int64_t l = 0; l < j; ++l) s -= Q[i + l * ldq] * Rp[l + j * n];
        Q[i + j * ldq] = s / Rp[j + j * n];
      }
    }
    if (Rp_out) memcpy(Rp_out, Rp, (size_t)(n * n) * sizeof(double));
  }
  free(Rp);
  free(G);
  free(Rs);
  return st;
}

/* Reverse-mode derivative of the thin QR with positive diagonal
 * (X = Q R, Q^T Q = I):  M = R dR^T - dQ^T Q,  N = copyltu(M) (the lower
 * triangle of M mirrored to the upper one),  dX = (dQ + Q N) R^{-T},
 * the last step by back substitution on each row (dx R^T = y).
 * The paper does not treat derivatives; this is the standard identity,
 * re-derived from d(QR) = dQ R + Q dR with Q^T dQ skew-symmetric. */
void orc_qr_backward(int64_t m, int64_t n, const double* Q, int64_t ldq,
                     const double* R, int64_t ldr, const double* dQ,
                     int64_t lddq, const double* dR, int64_t lddr, double* dX,
                     int64_t lddx) {
  double* M = (double*)malloc((size_t)(n * n) * sizeof(double));
  for (int64_t b = 0; b < n; ++b)
    for (int64_t a = 0; a < n; ++a) {
      /* (R dR^T)_{ab} = sum_l R_al dR_bl, over upper-triangular entries */
      double s = 0.0;
      for (int64_t l = 0; l < n; ++l) {
        double ra = (a <= l) ? R[a + l * ldr] : 0.0;
        double rb = (b <= l) ? dR[b + l * lddr] : 0.0;
        s += ra * rb;
      }
      double t = 0.0;
      for (int64_t i = 0; i < m; ++i) t += dQ[i + a * lddq] * Q[i + b * ldq];
      M[a + b * n] = s - t;
    }
  double* N = (double*)malloc((size_t)(n * n) * sizeof(double));
  for (int64_t b = 0; b < n; ++b)
    for (int64_t a = 0; a < n; ++a)
      N[a + b * n] = (a >= b) ? M[a + b * n] : M[b + a * n];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double y[4096];
    double* yp = (n <= 4096) ? y : (double*)malloc((size_t)n * sizeof(double));
    for (int64_t c = 0; c < n; ++c) {
      double s = dQ[i + c * lddq];
      for (int64_t l = 0; l < n; ++l) s += Q[i + l * ldq] * N[l + c * n];
      yp[c] = s;
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      double s = yp[j];
      for (int64_t l = j + 1; l < n; ++l) s -= dX[i + l * lddx] * R[j + l * ldr];
      dX[i + j * lddx] = s / R[j + j * ldr];
    }
    if (yp != y) free(yp);
  }
  free(N);
  free(M);
}

/* Number of threads the parallel loops above use (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
