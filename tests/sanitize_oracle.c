/* Driver of the CPU oracle for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py): tracks every
 * path of a small dense system with a work crew of several threads, runs the
 * duplicate scan, the double-double evaluation, refinement and residual, the
 * LU solve and the predictor, so that any out-of-bounds access, leak or
 * undefined operation on these paths aborts the run.  Exits 0 when all 12
 * paths converge and the scan finds no pair. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

/* a unit-circle coefficient from a linear congruential sequence */
static double lcg_angle(unsigned long long *state) {
  *state = *state * 6364136223846793005ULL + 1442695040888963407ULL;
  return 2.0 * M_PI * (double)(*state >> 11) / 9007199254740992.0;
}

int main(void) {
  /* n = 3, degrees (2, 3, 2): every monomial of degree <= d_i */
  enum { N = 3 };
  const int deg[N] = {2, 3, 2};
  int32_t eq_ptr[N + 1];
  uint8_t exps[64 * N];
  double coeff[2 * 64];
  unsigned long long st = 12345;
  int t = 0;
  eq_ptr[0] = 0;
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a <= deg[i]; ++a)
      for (int b = 0; a + b <= deg[i]; ++b)
        for (int c = 0; a + b + c <= deg[i]; ++c) {
          exps[t * N + 0] = (uint8_t)a;
          exps[t * N + 1] = (uint8_t)b;
          exps[t * N + 2] = (uint8_t)c;
          const double ang = lcg_angle(&st);
          coeff[2 * t] = cos(ang);
          coeff[2 * t + 1] = sin(ang);
          ++t;
        }
    eq_ptr[i + 1] = t;
  }
  ref_system f = {N, t, eq_ptr, coeff, exps};
  const double ang = lcg_angle(&st);
  const double gamma[2] = {cos(ang), sin(ang)};
  enum { P = 12 };
  double *ends = malloc(sizeof(double) * 2 * N * P);
  int32_t *status = malloc(sizeof(int32_t) * P);
  ref_path_stats *stats = malloc(sizeof(ref_path_stats) * P);
  ref_tolerances tol;
  ref_default_tolerances(&tol);
  if (ref_track_paths(&f, NULL, gamma, NULL, NULL, P, &tol, ends, status, stats, 4) != 0) return 2;
  int conv = 0;
  for (int p = 0; p < P; ++p) conv += status[p] == REF_CONVERGED;
  int64_t pairs[2 * 16];
  const int64_t np = ref_find_duplicates(N, P, ends, status, 1e-6, pairs, 16);
  double fh[2 * N], fl[2 * N], xr[2 * N], y[2 * N], jac[2 * N * N], fx[2 * N], xp[2 * N];
  ref_eval_system_dd(&f, ends, NULL, fh, fl);
  ref_refine_dd(&f, ends, 2, xr);
  double res[P];
  ref_residuals_dd(&f, P, ends, res);
  ref_eval_system(&f, ends, fx, jac);
  if (ref_lu_solve(N, jac, fx, y) != 0) return 3;
  if (ref_rk4_predict(&f, NULL, gamma, ends, 0.5, 0.01, xp) != 0) return 4;
  double sum[2], prod[2];
  ref_dd_ops(1.0, 1e-17, 3.0, -1e-17, sum, prod);
  printf("converged %d of %d, pairs %lld, residual %.3e\n", conv, P, (long long)np, res[0]);
  free(ends);
  free(status);
  free(stats);
  return (conv == P && np == 0) ? 0 : 1;
}
