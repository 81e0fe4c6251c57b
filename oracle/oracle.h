/*
 * CPU oracle for the batched homotopy path tracker -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this library.  The product path (the HIP library) never links, loads
 * or calls it, and this file shares no code with it.
 *
 * What it computes: the paths of the homotopy
 *     H(x,t) = gamma (1-t) g(x) + t f(x),   t in [0,1],
 * from the solutions of a start system g to the solutions of a square
 * polynomial system f.  The paper (Section 1 and the end of Section 2.1)
 * states only that these paths are tracked independently of each other
 * with no communication, with threads of a work crew pulling
 * jobs from a queue whose next-job pointer is guarded (Section 1).  It gives
 * no predictor, corrector or step control; the steps below are the reading
 * this project adopts (RK4 predictor on the Davidenko equation, Newton
 * corrector, halving/doubling step control, final Newton at t = 1).  The end
 * game refines the endpoint with Newton iterations whose residual is
 * evaluated in double-double arithmetic, rounds it to the nearest double,
 * and takes the residual test there, again in double-double: the endpoint
 * and the decision then no longer depend on the order of the double
 * precision arithmetic that led to them.
 *
 * Plain by design: every term and every partial derivative is evaluated by
 * repeated multiplication, the linear solver is textbook Gaussian
 * elimination with partial pivoting, complex division is Smith's method, and
 * the file is compiled with -ffp-contract=off.
 *
 * Complex vectors are interleaved (re, im) doubles.
 */
#ifndef HOMOTOPY_ORACLE_H
#define HOMOTOPY_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n;              /* unknowns == equations */
  int32_t n_terms;
  const int32_t *eq_ptr;  /* [n+1] CSR over equations */
  const double *coeff;    /* [2*n_terms] interleaved complex coefficients */
  const uint8_t *exps;    /* [n_terms*n] dense exponent vectors */
} ref_system;

typedef struct {
  double tol_residual; /* CONVERGED needs ||f(x)||_inf <= this at t = 1 */
  double tol_corr;     /* Newton corrector: ||dx|| <= tol_corr*max(1,||x||) */
  double tol_final;    /* final Newton at t = 1 stops at this relative size */
  double div_radius;   /* ||x||_inf above this: diverged (path truncated) */
  double h_init, h_min, h_max;
  int32_t max_steps, max_newton, max_newton_final;
} ref_tolerances;

/* Newton iterations in double-double at t = 1 after the double-precision
 * final Newton (see ref_refine_dd). */
#define REF_REFINE_ITERS 2

enum { REF_CONVERGED = 0, REF_DIVERGED = 1, REF_FAILED_MINSTEP = 2,
       REF_FAILED_MAXSTEPS = 3, REF_FAILED_NEWTON_T1 = 4 };

typedef struct {
  int32_t steps;        /* predictor-corrector attempts */
  int32_t rejections;   /* rejected attempts */
  int32_t newton_iters; /* corrector iterations, final Newton included */
  int32_t evals;        /* evaluations of H and its Jacobian */
  int32_t solves;       /* LU factorizations + solves */
  int32_t pad;
  double t_final;
  double residual;      /* ||f(x_end)||_inf */
} ref_path_stats;

void ref_default_tolerances(ref_tolerances *tol);

/* f(x) and its Jacobian, naive evaluation.  x: [2n], fx: [2n] (may be
 * NULL), jac: [2n*n] row-major (may be NULL). */
void ref_eval_system(const ref_system *s, const double *x, double *fx, double *jac);

/* Solves A y = b by LU with partial pivoting (largest |re|+|im| in the
 * column, ties to the lowest row).  A: [2n*n] row-major, b: [2n], y: [2n].
 * Returns 0, or -1 if a pivot is exactly zero. */
int ref_lu_solve(int n, const double *A, const double *b, double *y);

/* f(x) in double-double arithmetic at x = x_hi + x_lo (x_lo may be NULL):
 * [2n] interleaved complex each; f = f_hi + f_lo (f_lo may be NULL). */
void ref_eval_system_dd(const ref_system *s, const double *x_hi, const double *x_lo,
                        double *f_hi, double *f_lo);

/* ||f(x)||_inf at the double point x with f evaluated in double-double, each
 * |f_i| the modulus of the nearest complex double of f_i: the residual of
 * the end game. */
double ref_residual_dd(const ref_system *s, const double *x);
/* ref_residual_dd at each of the m points x[k*n .. k*n+n-1] (interleaved
 * complex) into out[k]. */
void ref_residuals_dd(const ref_system *s, int64_t m, const double *x, double *out);

/* End-game refinement: `iters` Newton iterations on f from x carried in
 * double-double (f in double-double, J_f and the solve in double), then the
 * nearest double of the result to x_out.  A zero pivot or a non-finite
 * update stops the iteration early. */
void ref_refine_dd(const ref_system *s, const double *x, int iters, double *x_out);

/* Double-double sum and product of a = a_hi + a_lo and b = b_hi + b_lo:
 * sum[2], prod[2] (hi, lo); for pinning the arithmetic. */
void ref_dd_ops(double a_hi, double a_lo, double b_hi, double b_lo, double *sum, double *prod);

/* Start point of a total-degree path: path id p is read in mixed radix,
 * p = sum_i k_i prod_{j<i} d_j (k_1 fastest), x_i = exp(2 pi i k_i/d_i). */
void ref_start_point(int n, const int32_t *degrees, int64_t path_id, double *x);

/* One RK4 predictor step (the tracker's predictor) from (x, t) with step
 * hstep; exported so tests can check its order against a closed-form path. */
int ref_rk4_predict(const ref_system *f, const ref_system *g, const double *gamma,
                    const double *x, double t, double hstep, double *xp);

/* Tracks paths of gamma(1-t) g + t f.
 *   g == NULL: total-degree start system g_i = x_i^{d_i} - 1, d_i = deg f_i.
 *   start == NULL: start points decoded from path ids (total degree only);
 *   otherwise start[2n*k] is the start point of the k-th tracked path.
 *   path_ids == NULL: tracks ids 0..n_paths-1; otherwise those ids.
 *   endpoints [2n*n_paths], status [n_paths], stats [n_paths] (nullable).
 *   n_threads: size of the work crew (atomic next-path counter).
 * Returns 0, or a negative value on invalid arguments. */
int ref_track_paths(const ref_system *f, const ref_system *g, const double *gamma,
                    const double *start, const int64_t *path_ids, int64_t n_paths,
                    const ref_tolerances *tol, double *endpoints, int32_t *status,
                    ref_path_stats *stats, int32_t n_threads);

/* The tracker of ref_track_paths with every operation on points, values,
 * Jacobians and linear systems in complex double-double (t and h in
 * double); the final Newton at t = 1 runs in double-double to tol_final and
 * the residual is ||f(x)||_inf with f in double-double.  Endpoints as
 * double-double pairs: ends_hi, ends_lo [2n*n_paths] each. */
int ref_track_paths_dd(const ref_system *f, const ref_system *g, const double *gamma,
                       const double *start, const int64_t *path_ids, int64_t n_paths,
                       const ref_tolerances *tol, double *ends_hi, double *ends_lo,
                       int32_t *status, ref_path_stats *stats, int32_t n_threads);

/* Pairs (a, b), a < b, of CONVERGED endpoints with
 * ||x_a - x_b||_inf <= rel * max(1, ||x_a||_inf), by comparing every pair.
 * Writes up to max_pairs pairs into pairs[2*k]; returns the pair count. */
int64_t ref_find_duplicates(int n, int64_t n_paths, const double *endpoints,
                            const int32_t *status, double rel, int64_t *pairs,
                            int64_t max_pairs);

#ifdef __cplusplus
}
#endif
#endif
