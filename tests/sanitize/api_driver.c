/* Host sanitizer driver for the library's host-side logic: workspace sizing
 * (every precision, kind and pass count over a grid of shapes) and the
 * synchronous argument checks of every entry point, none of which reaches a
 * GPU call.  Built against a copy of the library whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer; exit status 0 and no
 * sanitizer report is the pass condition. */
#include <stdint.h>
#include <stdio.h>

#include "rcholqr.h"

int main(void) {
  int failures = 0;
  const int64_t ms[] = {1, 17, 1000, 65537, 4000000, 100000000};
  const int64_t ns[] = {1, 16, 50, 200, 256, 257};
  size_t total = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b)
      for (int kind = 0; kind <= 3; ++kind)
        for (int passes = 1; passes <= 3; ++passes)
          for (int prec = 0; prec <= 3; ++prec) {
            const int64_t m = ms[a], n = ns[b];
            total += rcholqr_workspace_bytes(m, n, 3 * n, kind, passes, prec);
            total += rcholqr_reduced_workspace_bytes(m, n, 3 * n, n, kind, prec);
            total += rcholqr_rr_workspace_bytes(m, n, 3 * n, kind, prec, passes);
            total += rcholqr_col_block_workspace_bytes(m, n / 2, n - n / 2, 3 * n, kind, prec);
          }
  total += rcholqr_backward_workspace_bytes(1000, 64, 1);
  total += rcholqr_workspace_bytes(700, 40, 700, RCHOLQR_IDENTITY_TESTONLY, 1, RCHOLQR_F64);
  if (total == 0) ++failures;
  /* invalid arguments are refused before any launch */
  char buf[64];
  void* p = buf;
  double* d = (double*)buf;
  if (rcholqr_factor(p, 100, 0, 100, 10, 1, 0, 2, 0, p, 100, d, 1, NULL, 1, NULL, NULL, p,
                     1 << 30, NULL) != -3) ++failures;
  if (rcholqr_factor(p, 100, 10, 100, 5, 1, 0, 2, 0, p, 100, d, 10, NULL, 1, NULL, NULL, p,
                     1 << 30, NULL) != -5) ++failures;
  if (rcholqr_factor(p, 100, 10, 100, 30, 1, 0, 2, 0, p, 100, d, 10, NULL, 1, NULL, NULL, p,
                     16, NULL) != -19) ++failures;
  if (rcholqr_factor(p, 100, 10, 100, 99, 1, RCHOLQR_IDENTITY_TESTONLY, 1, 0, p, 100, d, 10,
                     NULL, 1, NULL, NULL, p, 1 << 30, NULL) != -5) ++failures;
  if (rcholqr_factor_noalloc(p, 4000000, 256, 4000000, 768, 1, 0, 2, 0, p, 4000000, d, 256,
                             NULL) != RCHOLQR_ERR_NOALLOC_SIZE) ++failures;
  rcholqr_problem pr = {p, 100, 10, 100, 5, 1, p, 100, d, 10};
  if (rcholqr_factor_batched(&pr, 1, 0, 2, 0, p, 1 << 30, NULL) != RCHOLQR_ERR_BATCH_ENTRY) ++failures;
  if (rcholqr_reduced(p, 100, 10, 100, 30, 0, 1, 0, 0, d, 1, d, 10, NULL, 1, p, 1 << 30, NULL) == 0)
    ++failures;
  if (rcholqr_rr(p, 100, 10, 100, 5, 1, 0, 0, 1, 1e-12, 0.0, p, 100, d, 10, (int*)p, (int*)p, p,
                 1 << 30, NULL) == 0) ++failures;
  if (rcholqr_col_block(p, 100, 0, 0, 100, 30, 1, 0, 0, p, 100, d, 30, d, 10, p, 1 << 30, NULL) == 0)
    ++failures;
  if (rcholqr_backward(p, 100, 0, 100, d, d, p, 100, d, 1, 0, p, 100, p, 1 << 30, NULL) == 0)
    ++failures;
  if (rcholqr_debug_theta(7, 10, 10, 1, 0, 1, 0, 1, d, NULL) == 0) ++failures;
  for (int code = -3001; code < 1100; code += 7) (void)rcholqr_error_string(code);
  printf("api driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
