/* Host sanitizer driver for the FP64 oracle (test infrastructure): runs each
 * exported oracle entry on small seeded inputs (every sketch kind, one and
 * two passes, a rank-deficient input, the Cholesky breakdown, the adjoint)
 * so that an AddressSanitizer / UndefinedBehaviorSanitizer build reports any
 * out-of-bounds access, leak or undefined operation.  Exit status 0 and no
 * sanitizer report is the pass condition. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double orc_ln(double x);
void orc_theta_block(int kind, int64_t k, int64_t m, uint64_t seed, int64_t i0, int64_t ni,
                     int64_t j0, int64_t nj, double* out);
void orc_countsketch_hash(int64_t k, uint64_t seed, int64_t j, int64_t* h, double* s);
void orc_sketch(int kind, int64_t m, int64_t n, int64_t k, uint64_t seed, const double* X,
                int64_t ldx, double* P, int64_t ldp);
int orc_householder_qr(int64_t k, int64_t n, const double* P, int64_t ldp, double* R,
                       int64_t ldr, double* S, int64_t lds);
int orc_cholesky_upper(int64_t n, const double* G, int64_t ldg, double* Rp, int64_t ldr);
int orc_rcholqr(int kind, int passes, int64_t m, int64_t n, int64_t k, uint64_t seed,
                const double* X, int64_t ldx, double* Q, int64_t ldq, double* R, int64_t ldr,
                double* S, int64_t lds, double* Rs_out, double* Rp_out);
void orc_qr_backward(int64_t m, int64_t n, const double* Q, int64_t ldq, const double* R,
                     int64_t ldr, const double* dQ, int64_t lddq, const double* dR,
                     int64_t lddr, double* dX, int64_t lddx);

/* xorshift64* uniform in (-1, 1): inputs only, no arithmetic of the method */
static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) {
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1p-52 - 1.0;
}

static double* filled(int64_t count) {
  double* a = (double*)malloc((size_t)count * sizeof(double));
  for (int64_t i = 0; i < count; ++i) a[i] = urand();
  return a;
}

int main(void) {
  int failures = 0;
  if (!(fabs(orc_ln(2.0) - 0.6931471805599453) < 1e-15)) ++failures;
  double theta[6 * 300];
  for (int kind = 0; kind <= 3; ++kind) orc_theta_block(kind, 6, 300, 7, 0, 6, 0, 300, theta);
  int64_t h;
  double sg;
  orc_countsketch_hash(30, 5, 12345, &h, &sg);
  if (h < 0 || h >= 30 || (sg != 1.0 && sg != -1.0)) ++failures;

  const int64_t m = 300, n = 7, k = 21;
  double* X = filled(m * n);
  double* Q = filled(m * n);
  double* R = filled(n * n);
  double* S = filled(k * n);
  double* Rs = filled(n * n);
  double* Rp = filled(n * n);
  double* P = filled(k * n);
  for (int kind = 0; kind <= 2; ++kind) {
    orc_sketch(kind, m, n, k, 3, X, m, P, k);
    if (orc_householder_qr(k, n, P, k, R, n, S, k) != 0) ++failures;
    for (int passes = 1; passes <= 2; ++passes)
      if (orc_rcholqr(kind, passes, m, n, k, 11, X, m, Q, m, R, n, S, k, Rs, Rp) != 0) ++failures;
  }
  /* identity kind: k = m */
  double* Pm = filled(m * n);
  orc_sketch(99, m, n, m, 0, X, m, Pm, m);
  /* a zero column: the sketch R has a zero diagonal (status 1) */
  double* Z = filled(m * n);
  for (int64_t i = 0; i < m; ++i) Z[i + 3 * m] = 0.0;
  if (orc_rcholqr(0, 1, m, n, k, 11, Z, m, Q, m, R, n, NULL, k, NULL, NULL) != 1) ++failures;
  /* Cholesky breakdown on an indefinite matrix */
  double G[9] = {1.0, 2.0, 0.0, 2.0, 1.0, 0.0, 0.0, 0.0, 1.0};
  double Rc[9];
  if (orc_cholesky_upper(3, G, 3, Rc, 3) == 0) ++failures;
  /* adjoint of the 2-pass factorisation */
  orc_rcholqr(0, 2, m, n, k, 11, X, m, Q, m, R, n, NULL, k, NULL, NULL);
  double* dQ = filled(m * n);
  double* dR = filled(n * n);
  double* dX = filled(m * n);
  orc_qr_backward(m, n, Q, m, R, n, dQ, m, dR, n, dX, m);
  for (int64_t i = 0; i < m * n; ++i)
    if (!isfinite(dX[i])) {
      ++failures;
      break;
    }
  free(X); free(Q); free(R); free(S); free(Rs); free(Rp); free(P); free(Pm); free(Z);
  free(dQ); free(dR); free(dX);
  printf("oracle driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
