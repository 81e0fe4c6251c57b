/*
 * CPU oracle for the batched homotopy path tracker -- TEST INFRASTRUCTURE.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it;
 * see oracle.h for the contract and the reading of the method it follows.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread oracle.c -lm
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define MAXN 16

void ref_default_tolerances(ref_tolerances *tol) {
  tol->tol_residual = 1e-10;
  tol->tol_corr = 1e-8;
  tol->tol_final = 1e-13;
  tol->div_radius = 1e8;
  tol->h_init = 0.01;
  tol->h_min = 1e-13;
  tol->h_max = 0.1;
  tol->max_steps = 10000;
  tol->max_newton = 3;
  tol->max_newton_final = 6;
}

static cplx load(const double *p, int i) { return CMPLX(p[2 * i], p[2 * i + 1]); }
static void store(double *p, int i, cplx z) { p[2 * i] = creal(z); p[2 * i + 1] = cimag(z); }

/* Smith's complex division a / b (Smith 1962). */
static cplx smith_div(cplx a, cplx b) {
  double ar = creal(a), ai = cimag(a), br = creal(b), bi = cimag(b);
  if (fabs(br) >= fabs(bi)) {
    double r = bi / br, den = br + bi * r;
    return CMPLX((ar + ai * r) / den, (ai - ar * r) / den);
  } else {
    double r = br / bi, den = br * r + bi;
    return CMPLX((ar * r + ai) / den, (ai * r - ar) / den);
  }
}

static double cabs1(cplx z) { return fabs(creal(z)) + fabs(cimag(z)); }

/* ||v||_inf with the complex modulus |z| = hypot(re, im). */
static double norm_inf(int n, const cplx *v) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) {
    double a = cabs(v[i]);
    if (!(a <= m)) m = a; /* also propagates NaN */
  }
  return m;
}

static int all_finite(int n, const cplx *v) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(creal(v[i])) || !isfinite(cimag(v[i]))) return 0;
  return 1;
}

/* ---------------------------------------------------------------------- */
/* Evaluation: f(x) and J_f(x) term by term, every monomial and every     */
/* partial derivative by repeated multiplication.                          */
/* ---------------------------------------------------------------------- */

static void eval_f(const ref_system *s, const cplx *x, cplx *fx, cplx *jac) {
  const int n = s->n;
  for (int i = 0; i < n; ++i) {
    if (fx) fx[i] = 0.0;
    if (jac)
      for (int j = 0; j < n; ++j) jac[i * n + j] = 0.0;
    for (int t = s->eq_ptr[i]; t < s->eq_ptr[i + 1]; ++t) {
      const uint8_t *a = s->exps + (size_t)t * n;
      cplx c = load(s->coeff, t);
      if (fx) {
        cplx v = c;
        for (int l = 0; l < n; ++l)
          for (int e = 0; e < a[l]; ++e) v = v * x[l];
        fx[i] += v;
      }
      if (jac) {
        /* d/dx_j (c x^a) = a_j c x^(a - e_j) */
        for (int j = 0; j < n; ++j) {
          if (a[j] == 0) continue;
          cplx v = c * (double)a[j];
          for (int l = 0; l < n; ++l) {
            int el = a[l] - (l == j ? 1 : 0);
            for (int e = 0; e < el; ++e) v = v * x[l];
          }
          jac[i * n + j] += v;
        }
      }
    }
  }
}

void ref_eval_system(const ref_system *s, const double *x, double *fx, double *jac) {
  const int n = s->n;
  cplx xv[MAXN], fv[MAXN], jv[MAXN * MAXN];
  for (int i = 0; i < n; ++i) xv[i] = load(x, i);
  eval_f(s, xv, fx ? fv : NULL, jac ? jv : NULL);
  if (fx)
    for (int i = 0; i < n; ++i) store(fx, i, fv[i]);
  if (jac)
    for (int i = 0; i < n * n; ++i) store(jac, i, jv[i]);
}

/* ---------------------------------------------------------------------- */
/* Linear solve: Gaussian elimination with partial pivoting (outer product */
/* form), then forward and back substitution.                              */
/* ---------------------------------------------------------------------- */

static int lu_solve(int n, cplx *A, const cplx *b, cplx *y) {
  int piv[MAXN];
  for (int k = 0; k < n; ++k) {
    int mu = k;
    double best = cabs1(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = cabs1(A[i * n + k]);
      if (v > best) { best = v; mu = i; } /* strict: ties keep the lowest row */
    }
    piv[k] = mu;
    if (mu != k)
      for (int j = 0; j < n; ++j) {
        cplx tmp = A[k * n + j]; A[k * n + j] = A[mu * n + j]; A[mu * n + j] = tmp;
      }
    cplx p = A[k * n + k];
    if (creal(p) == 0.0 && cimag(p) == 0.0) return -1;
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] = smith_div(A[i * n + k], p);
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= A[i * n + k] * A[k * n + j];
    }
  }
  cplx z[MAXN];
  for (int i = 0; i < n; ++i) z[i] = b[i];
  for (int k = 0; k < n; ++k) {
    cplx tmp = z[k]; z[k] = z[piv[k]]; z[piv[k]] = tmp;
  }
  for (int i = 0; i < n; ++i) /* L z = P b, unit lower triangular */
    for (int j = 0; j < i; ++j) z[i] -= A[i * n + j] * z[j];
  for (int i = n - 1; i >= 0; --i) { /* U y = z */
    cplx v = z[i];
    for (int j = i + 1; j < n; ++j) v -= A[i * n + j] * y[j];
    y[i] = smith_div(v, A[i * n + i]);
  }
  return 0;
}

int ref_lu_solve(int n, const double *A, const double *b, double *y) {
  if (n < 1 || n > MAXN) return -2;
  cplx Av[MAXN * MAXN], bv[MAXN], yv[MAXN];
  for (int i = 0; i < n * n; ++i) Av[i] = load(A, i);
  for (int i = 0; i < n; ++i) bv[i] = load(b, i);
  int rc = lu_solve(n, Av, bv, yv);
  for (int i = 0; i < n; ++i) store(y, i, yv[i]);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Double-double arithmetic for the end game: a value is hi + lo with      */
/* |lo| <= ulp(hi)/2.  Error-free transformations: Knuth's two-sum and the  */
/* exact product from a fused multiply-add (C99 fma rounds once).          */
/* ---------------------------------------------------------------------- */

typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } cdd;

/* s + e == a + b exactly, s = fl(a + b) (Knuth, TAOCP vol. 2, 4.2.2) */
static dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  dd r = {s, e};
  return r;
}

/* s + e == a + b exactly when |a| >= |b| or a == 0 (Dekker) */
static dd fast_two_sum(double a, double b) {
  double s = a + b;
  dd r = {s, b - (s - a)};
  return r;
}

/* p + e == a * b exactly */
static dd two_prod(double a, double b) {
  double p = a * b;
  dd r = {p, fma(a, b, -p)};
  return r;
}

static dd dd_from(double a) { dd r = {a, 0.0}; return r; }

/* (a.hi + a.lo) + (b.hi + b.lo): both high parts and both low parts are
 * summed error-free, then renormalised */
static dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

static dd dd_neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }

/* (a.hi + a.lo)(b.hi + b.lo) without the lo*lo term */
static dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}

static cdd cdd_from(cplx z) { cdd r = {dd_from(creal(z)), dd_from(cimag(z))}; return r; }

static cdd cdd_add(cdd a, cdd b) {
  cdd r = {dd_add(a.re, b.re), dd_add(a.im, b.im)};
  return r;
}

static cdd cdd_mul(cdd a, cdd b) {
  cdd r = {dd_add(dd_mul(a.re, b.re), dd_neg(dd_mul(a.im, b.im))),
           dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
  return r;
}

/* the nearest complex double of z */
static cplx cdd_round(cdd z) { return CMPLX(z.re.hi + z.re.lo, z.im.hi + z.im.lo); }

/* f(x) in double-double at the double-double point x: every term by
 * repeated multiplication, summed per equation */
static void eval_f_dd(const ref_system *s, const cdd *x, cdd *fx) {
  const int n = s->n;
  for (int i = 0; i < n; ++i) {
    cdd acc = cdd_from(0.0);
    for (int t = s->eq_ptr[i]; t < s->eq_ptr[i + 1]; ++t) {
      const uint8_t *a = s->exps + (size_t)t * n;
      cdd v = cdd_from(load(s->coeff, t));
      for (int l = 0; l < n; ++l)
        for (int e = 0; e < a[l]; ++e) v = cdd_mul(v, x[l]);
      acc = cdd_add(acc, v);
    }
    fx[i] = acc;
  }
}

/* ||f(x)||_inf at the double point x, with f evaluated in double-double
 * and each |f_i| taken of its nearest complex double */
static double residual_dd(const ref_system *s, const cplx *x) {
  const int n = s->n;
  cdd xv[MAXN], fv[MAXN];
  cplx fr[MAXN];
  for (int i = 0; i < n; ++i) xv[i] = cdd_from(x[i]);
  eval_f_dd(s, xv, fv);
  for (int i = 0; i < n; ++i) fr[i] = cdd_round(fv[i]);
  return norm_inf(n, fr);
}

/* Newton refinement at t = 1 with the residual in double-double: x is
 * carried as a double-double point, each iteration solves J_f(x) d = f(x)
 * in double (J_f at the double part of x, f rounded to double) and
 * subtracts d in double-double.  Stops early on a zero pivot or a
 * non-finite update (x is kept).  On return x holds the nearest double of
 * the refined point. */
static void refine_dd(const ref_system *s, cplx *x, int iters) {
  const int n = s->n;
  cdd xv[MAXN], fv[MAXN];
  for (int i = 0; i < n; ++i) xv[i] = cdd_from(x[i]);
  for (int it = 0; it < iters; ++it) {
    cplx xh[MAXN], J[MAXN * MAXN], r[MAXN], d[MAXN];
    for (int i = 0; i < n; ++i) xh[i] = cdd_round(xv[i]);
    eval_f_dd(s, xv, fv);
    for (int i = 0; i < n; ++i) r[i] = cdd_round(fv[i]);
    eval_f(s, xh, NULL, J);
    if (lu_solve(n, J, r, d) != 0 || !all_finite(n, d)) break;
    for (int i = 0; i < n; ++i) xv[i] = cdd_add(xv[i], cdd_from(-d[i]));
  }
  for (int i = 0; i < n; ++i) x[i] = cdd_round(xv[i]);
}

void ref_eval_system_dd(const ref_system *s, const double *x_hi, const double *x_lo,
                        double *f_hi, double *f_lo) {
  const int n = s->n;
  cdd xv[MAXN], fv[MAXN];
  for (int i = 0; i < n; ++i) {
    xv[i].re = fast_two_sum(x_hi[2 * i], x_lo ? x_lo[2 * i] : 0.0);
    xv[i].im = fast_two_sum(x_hi[2 * i + 1], x_lo ? x_lo[2 * i + 1] : 0.0);
  }
  eval_f_dd(s, xv, fv);
  for (int i = 0; i < n; ++i) {
    f_hi[2 * i] = fv[i].re.hi;
    f_hi[2 * i + 1] = fv[i].im.hi;
    if (f_lo) {
      f_lo[2 * i] = fv[i].re.lo;
      f_lo[2 * i + 1] = fv[i].im.lo;
    }
  }
}

double ref_residual_dd(const ref_system *s, const double *x) {
  cplx xv[MAXN];
  for (int i = 0; i < s->n; ++i) xv[i] = load(x, i);
  return residual_dd(s, xv);
}

void ref_residuals_dd(const ref_system *s, int64_t m, const double *x, double *out) {
  for (int64_t k = 0; k < m; ++k) out[k] = ref_residual_dd(s, x + (size_t)2 * s->n * k);
}

void ref_refine_dd(const ref_system *s, const double *x, int iters, double *x_out) {
  cplx xv[MAXN];
  for (int i = 0; i < s->n; ++i) xv[i] = load(x, i);
  refine_dd(s, xv, iters);
  for (int i = 0; i < s->n; ++i) store(x_out, i, xv[i]);
}

void ref_dd_ops(double a_hi, double a_lo, double b_hi, double b_lo, double *sum, double *prod) {
  dd a = fast_two_sum(a_hi, a_lo), b = fast_two_sum(b_hi, b_lo);
  dd s = dd_add(a, b), p = dd_mul(a, b);
  sum[0] = s.hi; sum[1] = s.lo;
  prod[0] = p.hi; prod[1] = p.lo;
}

/* ---------------------------------------------------------------------- */
/* Homotopy H(x,t) = gamma (1-t) g(x) + t f(x)                              */
/* ---------------------------------------------------------------------- */

typedef struct {
  const ref_system *f, *g; /* g == NULL: total degree */
  int n;
  int32_t deg[MAXN];
  cplx gamma;
} homotopy;

static void eval_g(const homotopy *h, const cplx *x, cplx *gx, cplx *jg) {
  const int n = h->n;
  if (h->g) { eval_f(h->g, x, gx, jg); return; }
  for (int i = 0; i < n; ++i) { /* g_i = x_i^{d_i} - 1, dg_i/dx_i = d_i x_i^{d_i-1} */
    cplx p = 1.0;
    for (int e = 0; e < h->deg[i] - 1; ++e) p = p * x[i];
    if (gx) gx[i] = p * x[i] - 1.0;
    if (jg) {
      for (int j = 0; j < n; ++j) jg[i * n + j] = 0.0;
      jg[i * n + i] = (double)h->deg[i] * p;
    }
  }
}

/* H and J_x at (x, t); Ht = dH/dt = f - gamma g (any of the outputs may be NULL). */
static void eval_h(const homotopy *h, const cplx *x, double t, cplx *H, cplx *Jx, cplx *Ht) {
  const int n = h->n;
  cplx fx[MAXN], gx[MAXN], jf[MAXN * MAXN], jg[MAXN * MAXN];
  eval_f(h->f, x, fx, Jx ? jf : NULL);
  eval_g(h, x, gx, Jx ? jg : NULL);
  cplx s = h->gamma * (1.0 - t);
  for (int i = 0; i < n; ++i) {
    if (H) H[i] = s * gx[i] + t * fx[i];
    if (Ht) Ht[i] = fx[i] - h->gamma * gx[i];
  }
  if (Jx)
    for (int i = 0; i < n * n; ++i) Jx[i] = t * jf[i] + s * jg[i];
}

/* ---------------------------------------------------------------------- */
/* One path                                                                 */
/* ---------------------------------------------------------------------- */

void ref_start_point(int n, const int32_t *degrees, int64_t path_id, double *x) {
  int64_t p = path_id;
  for (int i = 0; i < n; ++i) {
    int64_t k = p % degrees[i];
    p /= degrees[i];
    double ang = 2.0 * M_PI * (double)k / (double)degrees[i];
    x[2 * i] = cos(ang);
    x[2 * i + 1] = sin(ang);
  }
}

/* Davidenko direction dx/dt = -J_x^{-1} H_t at (x, t). */
static int tangent(const homotopy *h, const cplx *x, double t, cplx *k, ref_path_stats *st) {
  const int n = h->n;
  cplx J[MAXN * MAXN], Ht[MAXN], rhs[MAXN];
  eval_h(h, x, t, NULL, J, Ht);
  st->evals++;
  for (int i = 0; i < n; ++i) rhs[i] = -Ht[i];
  st->solves++;
  if (lu_solve(n, J, rhs, k) != 0) return -1;
  return all_finite(n, k) ? 0 : -1;
}

/* Classical fourth-order Runge-Kutta step for the Davidenko equation
 * dx/dt = -J_x^{-1} H_t from (x, t) with step hstep to t_new = t + hstep;
 * each stage is a fresh evaluation and solve. */
static int rk4_predict(const homotopy *h, const cplx *x, double t, double hstep, double t_new,
                       cplx *xp, ref_path_stats *st) {
  const int n = h->n;
  cplx xs[MAXN], k1[MAXN], k2[MAXN], k3[MAXN], k4[MAXN];
  double th = t + 0.5 * hstep;
  if (tangent(h, x, t, k1, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = x[i] + (0.5 * hstep) * k1[i];
  if (tangent(h, xs, th, k2, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = x[i] + (0.5 * hstep) * k2[i];
  if (tangent(h, xs, th, k3, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = x[i] + hstep * k3[i];
  if (tangent(h, xs, t_new, k4, st) != 0) return -1;
  for (int i = 0; i < n; ++i)
    xp[i] = x[i] + (hstep / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  return all_finite(n, xp) ? 0 : -1;
}

/* Newton on H(., t) from x (in place).  Succeeds when the update satisfies
 * ||dx|| <= tol * max(1, ||x||) (x after the update); fails on a zero
 * pivot, a non-finite value, no contraction (||dx_j|| > ||dx_{j-1}||/2 from
 * the second iteration on), or when max_it iterations do not succeed. */
static int newton(const homotopy *h, cplx *x, double t, int max_it, double tol,
                  int check_contraction, ref_path_stats *st) {
  const int n = h->n;
  double prev = 0.0;
  for (int it = 1; it <= max_it; ++it) {
    cplx J[MAXN * MAXN], H[MAXN], dx[MAXN];
    eval_h(h, x, t, H, J, NULL);
    st->evals++;
    st->solves++;
    st->newton_iters++;
    if (lu_solve(n, J, H, dx) != 0) return 0;
    for (int i = 0; i < n; ++i) x[i] -= dx[i];
    if (!all_finite(n, dx) || !all_finite(n, x)) return 0;
    double nd = norm_inf(n, dx);
    double nx = norm_inf(n, x);
    if (nd <= tol * (nx > 1.0 ? nx : 1.0)) return 1;
    if (check_contraction && it >= 2 && nd > 0.5 * prev) return 0;
    prev = nd;
  }
  return 0;
}

static void track_one(const homotopy *h, const cplx *x_start, const ref_tolerances *tol,
                      cplx *x_end, int32_t *status, ref_path_stats *st) {
  const int n = h->n;
  cplx x[MAXN], xp[MAXN];
  memset(st, 0, sizeof(*st));
  for (int i = 0; i < n; ++i) x[i] = x_start[i];
  double t = 0.0, hstep = tol->h_init;
  int accepts = 0;
  int32_t stat = -1;

  while (t < 1.0) {
    /* step size, clipped so the step ends exactly at t = 1 */
    double t_new;
    if (hstep >= 1.0 - t) { hstep = 1.0 - t; t_new = 1.0; }
    else t_new = t + hstep;

    /* RK4 predictor on dx/dt = -J_x^{-1} H_t */
    int ok = rk4_predict(h, x, t, hstep, t_new, xp, st) == 0;
    /* Newton corrector at t_new */
    if (ok) ok = newton(h, xp, t_new, tol->max_newton, tol->tol_corr, 1, st);

    st->steps++;
    if (ok) {
      t = t_new;
      for (int i = 0; i < n; ++i) x[i] = xp[i];
      if (++accepts == 3) {
        hstep = 2.0 * hstep < tol->h_max ? 2.0 * hstep : tol->h_max;
        accepts = 0;
      }
    } else {
      st->rejections++;
      hstep = 0.5 * hstep;
      accepts = 0;
    }
    if (norm_inf(n, x) > tol->div_radius) { stat = REF_DIVERGED; break; }
    if (t >= 1.0) break; /* reached t = 1: the step-size tests no longer apply */
    if (hstep < tol->h_min) { stat = REF_FAILED_MINSTEP; break; }
    if (st->steps > tol->max_steps) { stat = REF_FAILED_MAXSTEPS; break; }
  }

  if (stat < 0) {
    /* t = 1: Newton on f = H(., 1) without the contraction test, then the
     * double-double refinement to the nearest double of the root and the
     * residual there, evaluated in double-double: two implementations that
     * differ in rounding reach the same endpoint and the same decision */
    newton(h, x, 1.0, tol->max_newton_final, tol->tol_final, 0, st);
    double nx = norm_inf(n, x);
    double res;
    if (all_finite(n, x) && nx <= tol->div_radius) {
      refine_dd(h->f, x, REF_REFINE_ITERS);
      nx = norm_inf(n, x);
      res = residual_dd(h->f, x);
    } else {
      cplx fx[MAXN];
      eval_f(h->f, x, fx, NULL);
      res = norm_inf(n, fx);
    }
    st->residual = res;
    if (res <= tol->tol_residual && nx <= tol->div_radius) stat = REF_CONVERGED;
    else if (nx > tol->div_radius) stat = REF_DIVERGED;
    else stat = REF_FAILED_NEWTON_T1;
  } else {
    cplx fx[MAXN];
    eval_f(h->f, x, fx, NULL);
    st->residual = norm_inf(n, fx);
  }
  st->t_final = t;
  for (int i = 0; i < n; ++i) x_end[i] = x[i];
  *status = stat;
}

static int make_homotopy(const ref_system *f, const ref_system *g, const double *gamma,
                         homotopy *h) {
  memset(h, 0, sizeof(*h));
  h->f = f;
  h->g = g;
  h->n = f->n;
  h->gamma = CMPLX(gamma[0], gamma[1]);
  for (int i = 0; i < f->n; ++i) {
    int d = 0;
    for (int t = f->eq_ptr[i]; t < f->eq_ptr[i + 1]; ++t) {
      int s = 0;
      for (int l = 0; l < f->n; ++l) s += f->exps[(size_t)t * f->n + l];
      if (s > d) d = s;
    }
    if (d < 1) return -1;
    h->deg[i] = d;
  }
  return 0;
}

int ref_rk4_predict(const ref_system *f, const ref_system *g, const double *gamma,
                    const double *x, double t, double hstep, double *xp) {
  if (!f || f->n < 1 || f->n > MAXN) return -1;
  homotopy h;
  if (make_homotopy(f, g, gamma, &h) != 0) return -1;
  cplx xv[MAXN], pv[MAXN];
  for (int i = 0; i < f->n; ++i) xv[i] = load(x, i);
  ref_path_stats st;
  memset(&st, 0, sizeof(st));
  int rc = rk4_predict(&h, xv, t, hstep, t + hstep, pv, &st);
  for (int i = 0; i < f->n; ++i) store(xp, i, pv[i]);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Work crew: threads pull path indices from an atomic next-job counter.   */
/* ---------------------------------------------------------------------- */

typedef struct {
  const homotopy *h;
  const double *start;
  const int64_t *ids;
  int64_t n_paths;
  const ref_tolerances *tol;
  double *endpoints;
  int32_t *status;
  ref_path_stats *stats;
  atomic_llong next;
} crew;

static void *crew_worker(void *arg) {
  crew *c = (crew *)arg;
  const int n = c->h->n;
  for (;;) {
    int64_t k = atomic_fetch_add(&c->next, 1);
    if (k >= c->n_paths) break;
    cplx xs[MAXN], xe[MAXN];
    if (c->start) {
      for (int i = 0; i < n; ++i) xs[i] = load(c->start + (size_t)2 * n * k, i);
    } else {
      double tmp[2 * MAXN];
      ref_start_point(n, c->h->deg, c->ids ? c->ids[k] : k, tmp);
      for (int i = 0; i < n; ++i) xs[i] = load(tmp, i);
    }
    ref_path_stats st;
    int32_t s;
    track_one(c->h, xs, c->tol, xe, &s, &st);
    for (int i = 0; i < n; ++i) store(c->endpoints + (size_t)2 * n * k, i, xe[i]);
    c->status[k] = s;
    if (c->stats) c->stats[k] = st;
  }
  return NULL;
}

int ref_track_paths(const ref_system *f, const ref_system *g, const double *gamma,
                    const double *start, const int64_t *path_ids, int64_t n_paths,
                    const ref_tolerances *tol, double *endpoints, int32_t *status,
                    ref_path_stats *stats, int32_t n_threads) {
  if (!f || f->n < 1 || f->n > MAXN || n_paths < 0 || !endpoints || !status) return -1;
  if (g && g->n != f->n) return -1;
  if (g && !start) return -1;
  ref_tolerances deftol;
  if (!tol) { ref_default_tolerances(&deftol); tol = &deftol; }
  homotopy h;
  if (make_homotopy(f, g, gamma, &h) != 0) return -1;
  crew c;
  c.h = &h;
  c.start = start;
  c.ids = path_ids;
  c.n_paths = n_paths;
  c.tol = tol;
  c.endpoints = endpoints;
  c.status = status;
  c.stats = stats;
  atomic_init(&c.next, 0);
  if (n_threads < 1) n_threads = 1;
  if (n_threads == 1) {
    crew_worker(&c);
    return 0;
  }
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -3;
  int started = 0;
  for (int i = 0; i < n_threads; ++i)
    if (pthread_create(&th[i], NULL, crew_worker, &c) == 0) ++started;
  if (started == 0) crew_worker(&c);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  return 0;
}

int64_t ref_find_duplicates(int n, int64_t n_paths, const double *endpoints,
                            const int32_t *status, double rel, int64_t *pairs,
                            int64_t max_pairs) {
  int64_t count = 0;
  for (int64_t a = 0; a < n_paths; ++a) {
    if (status[a] != REF_CONVERGED) continue;
    cplx xa[MAXN];
    for (int i = 0; i < n; ++i) xa[i] = load(endpoints + (size_t)2 * n * a, i);
    double scale = norm_inf(n, xa);
    if (scale < 1.0) scale = 1.0;
    for (int64_t b = a + 1; b < n_paths; ++b) {
      if (status[b] != REF_CONVERGED) continue;
      cplx d[MAXN];
      for (int i = 0; i < n; ++i) d[i] = load(endpoints + (size_t)2 * n * b, i) - xa[i];
      if (norm_inf(n, d) <= rel * scale) {
        if (count < max_pairs) { pairs[2 * count] = a; pairs[2 * count + 1] = b; }
        ++count;
      }
    }
  }
  return count;
}

/* ---------------------------------------------------------------------- */
/* Double-double tracker: the same homotopy, predictor, corrector, step    */
/* control and end game as track_one, every operation on points, function  */
/* values, Jacobians and linear systems in complex double-double (the      */
/* paper's "quality up": Section 1, Section 5.1 and Table 2 track in       */
/* double-double).  t and h stay doubles: the path parameter and the step  */
/* size are exact in double.  Norms and the tests on them use the nearest  */
/* double of each double-double value.                                     */
/* ---------------------------------------------------------------------- */

static dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

/* a / b: three quotient digits, each from the remainder (Dekker-style long
 * division in double-double) */
static dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul(b, dd_from(q1)));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul(b, dd_from(q2)));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd_from(q3));
}

static double dd_to(dd a) { return a.hi + a.lo; }

static cdd cdd_sub(cdd a, cdd b) {
  cdd r = {dd_sub(a.re, b.re), dd_sub(a.im, b.im)};
  return r;
}

static cdd cdd_scale(cdd a, double s) {
  cdd r = {dd_mul(a.re, dd_from(s)), dd_mul(a.im, dd_from(s))};
  return r;
}

/* Smith's division in double-double */
static cdd cdd_div(cdd a, cdd b) {
  cdd q;
  if (fabs(dd_to(b.re)) >= fabs(dd_to(b.im))) {
    dd r = dd_div(b.im, b.re);
    dd den = dd_add(b.re, dd_mul(b.im, r));
    q.re = dd_div(dd_add(a.re, dd_mul(a.im, r)), den);
    q.im = dd_div(dd_sub(a.im, dd_mul(a.re, r)), den);
  } else {
    dd r = dd_div(b.re, b.im);
    dd den = dd_add(dd_mul(b.re, r), b.im);
    q.re = dd_div(dd_add(dd_mul(a.re, r), a.im), den);
    q.im = dd_div(dd_sub(dd_mul(a.im, r), a.re), den);
  }
  return q;
}

static double cdd_abs(cdd z) { return cabs(cdd_round(z)); }
static double cdd_abs1(cdd z) { return fabs(dd_to(z.re)) + fabs(dd_to(z.im)); }
static int cdd_finite(cdd z) { return isfinite(dd_to(z.re)) && isfinite(dd_to(z.im)); }

static double norm_inf_dd(int n, const cdd *v) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) {
    double a = cdd_abs(v[i]);
    if (!(a <= m)) m = a;
  }
  return m;
}

static int all_finite_dd(int n, const cdd *v) {
  for (int i = 0; i < n; ++i)
    if (!cdd_finite(v[i])) return 0;
  return 1;
}

/* f(x) and J_f(x) in double-double: terms and partial derivatives by
 * repeated multiplication, as eval_f */
static void eval_f_ddj(const ref_system *s, const cdd *x, cdd *fx, cdd *jac) {
  const int n = s->n;
  const cdd zero = cdd_from(0.0);
  for (int i = 0; i < n; ++i) {
    if (fx) fx[i] = zero;
    if (jac)
      for (int j = 0; j < n; ++j) jac[i * n + j] = zero;
    for (int t = s->eq_ptr[i]; t < s->eq_ptr[i + 1]; ++t) {
      const uint8_t *a = s->exps + (size_t)t * n;
      cdd c = cdd_from(load(s->coeff, t));
      if (fx) {
        cdd v = c;
        for (int l = 0; l < n; ++l)
          for (int e = 0; e < a[l]; ++e) v = cdd_mul(v, x[l]);
        fx[i] = cdd_add(fx[i], v);
      }
      if (jac)
        for (int j = 0; j < n; ++j) {
          if (a[j] == 0) continue;
          cdd v = cdd_scale(c, (double)a[j]);
          for (int l = 0; l < n; ++l) {
            int el = a[l] - (l == j ? 1 : 0);
            for (int e = 0; e < el; ++e) v = cdd_mul(v, x[l]);
          }
          jac[i * n + j] = cdd_add(jac[i * n + j], v);
        }
    }
  }
}

static void eval_g_dd(const homotopy *h, const cdd *x, cdd *gx, cdd *jg) {
  const int n = h->n;
  if (h->g) { eval_f_ddj(h->g, x, gx, jg); return; }
  for (int i = 0; i < n; ++i) {
    cdd p = cdd_from(1.0);
    for (int e = 0; e < h->deg[i] - 1; ++e) p = cdd_mul(p, x[i]);
    if (gx) gx[i] = cdd_sub(cdd_mul(p, x[i]), cdd_from(1.0));
    if (jg) {
      for (int j = 0; j < n; ++j) jg[i * n + j] = cdd_from(0.0);
      jg[i * n + i] = cdd_scale(p, (double)h->deg[i]);
    }
  }
}

/* H, J_x and H_t at (x, t) in double-double (outputs may be NULL) */
static void eval_h_dd(const homotopy *h, const cdd *x, double t, cdd *H, cdd *Jx, cdd *Ht) {
  const int n = h->n;
  cdd fx[MAXN], gx[MAXN], jf[MAXN * MAXN], jg[MAXN * MAXN];
  eval_f_ddj(h->f, x, fx, Jx ? jf : NULL);
  eval_g_dd(h, x, gx, Jx ? jg : NULL);
  const cdd gam = cdd_from(h->gamma);
  const cdd s = cdd_scale(gam, 1.0 - t);
  for (int i = 0; i < n; ++i) {
    if (H) H[i] = cdd_add(cdd_mul(s, gx[i]), cdd_scale(fx[i], t));
    if (Ht) Ht[i] = cdd_sub(fx[i], cdd_mul(gam, gx[i]));
  }
  if (Jx)
    for (int i = 0; i < n * n; ++i) Jx[i] = cdd_add(cdd_scale(jf[i], t), cdd_mul(s, jg[i]));
}

/* LU with partial pivoting (largest |re| + |im| of the nearest double, ties
 * to the lowest row) and the two triangular solves, in double-double */
static int lu_solve_dd(int n, cdd *A, const cdd *b, cdd *y) {
  int piv[MAXN];
  for (int k = 0; k < n; ++k) {
    int mu = k;
    double best = cdd_abs1(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = cdd_abs1(A[i * n + k]);
      if (v > best) { best = v; mu = i; }
    }
    piv[k] = mu;
    if (mu != k)
      for (int j = 0; j < n; ++j) {
        cdd tmp = A[k * n + j]; A[k * n + j] = A[mu * n + j]; A[mu * n + j] = tmp;
      }
    cdd p = A[k * n + k];
    if (dd_to(p.re) == 0.0 && dd_to(p.im) == 0.0) return -1;
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] = cdd_div(A[i * n + k], p);
      for (int j = k + 1; j < n; ++j)
        A[i * n + j] = cdd_sub(A[i * n + j], cdd_mul(A[i * n + k], A[k * n + j]));
    }
  }
  cdd z[MAXN];
  for (int i = 0; i < n; ++i) z[i] = b[i];
  for (int k = 0; k < n; ++k) {
    cdd tmp = z[k]; z[k] = z[piv[k]]; z[piv[k]] = tmp;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) z[i] = cdd_sub(z[i], cdd_mul(A[i * n + j], z[j]));
  for (int i = n - 1; i >= 0; --i) {
    cdd v = z[i];
    for (int j = i + 1; j < n; ++j) v = cdd_sub(v, cdd_mul(A[i * n + j], y[j]));
    y[i] = cdd_div(v, A[i * n + i]);
  }
  return 0;
}

static int tangent_dd(const homotopy *h, const cdd *x, double t, cdd *k, ref_path_stats *st) {
  const int n = h->n;
  cdd J[MAXN * MAXN], Ht[MAXN], rhs[MAXN];
  eval_h_dd(h, x, t, NULL, J, Ht);
  st->evals++;
  for (int i = 0; i < n; ++i) rhs[i] = cdd_scale(Ht[i], -1.0);
  st->solves++;
  if (lu_solve_dd(n, J, rhs, k) != 0) return -1;
  return all_finite_dd(n, k) ? 0 : -1;
}

static int rk4_predict_dd(const homotopy *h, const cdd *x, double t, double hstep, double t_new,
                          cdd *xp, ref_path_stats *st) {
  const int n = h->n;
  cdd xs[MAXN], k1[MAXN], k2[MAXN], k3[MAXN], k4[MAXN];
  const double th = t + 0.5 * hstep;
  if (tangent_dd(h, x, t, k1, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = cdd_add(x[i], cdd_scale(k1[i], 0.5 * hstep));
  if (tangent_dd(h, xs, th, k2, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = cdd_add(x[i], cdd_scale(k2[i], 0.5 * hstep));
  if (tangent_dd(h, xs, th, k3, st) != 0) return -1;
  for (int i = 0; i < n; ++i) xs[i] = cdd_add(x[i], cdd_scale(k3[i], hstep));
  if (tangent_dd(h, xs, t_new, k4, st) != 0) return -1;
  for (int i = 0; i < n; ++i) {
    cdd sum = cdd_add(cdd_add(k1[i], cdd_scale(k2[i], 2.0)), cdd_add(cdd_scale(k3[i], 2.0), k4[i]));
    xp[i] = cdd_add(x[i], cdd_scale(sum, hstep / 6.0));
  }
  return all_finite_dd(n, xp) ? 0 : -1;
}

static int newton_dd(const homotopy *h, cdd *x, double t, int max_it, double tol,
                     int check_contraction, ref_path_stats *st) {
  const int n = h->n;
  double prev = 0.0;
  for (int it = 1; it <= max_it; ++it) {
    cdd J[MAXN * MAXN], H[MAXN], dx[MAXN];
    eval_h_dd(h, x, t, H, J, NULL);
    st->evals++;
    st->solves++;
    st->newton_iters++;
    if (lu_solve_dd(n, J, H, dx) != 0) return 0;
    for (int i = 0; i < n; ++i) x[i] = cdd_sub(x[i], dx[i]);
    if (!all_finite_dd(n, dx) || !all_finite_dd(n, x)) return 0;
    double nd = norm_inf_dd(n, dx);
    double nx = norm_inf_dd(n, x);
    if (nd <= tol * (nx > 1.0 ? nx : 1.0)) return 1;
    if (check_contraction && it >= 2 && nd > 0.5 * prev) return 0;
    prev = nd;
  }
  return 0;
}

static void track_one_dd(const homotopy *h, const cplx *x_start, const ref_tolerances *tol,
                         cdd *x_end, int32_t *status, ref_path_stats *st) {
  const int n = h->n;
  cdd x[MAXN], xp[MAXN];
  memset(st, 0, sizeof(*st));
  for (int i = 0; i < n; ++i) x[i] = cdd_from(x_start[i]);
  double t = 0.0, hstep = tol->h_init;
  int accepts = 0;
  int32_t stat = -1;
  while (t < 1.0) {
    double t_new;
    if (hstep >= 1.0 - t) { hstep = 1.0 - t; t_new = 1.0; }
    else t_new = t + hstep;
    int ok = rk4_predict_dd(h, x, t, hstep, t_new, xp, st) == 0;
    if (ok) ok = newton_dd(h, xp, t_new, tol->max_newton, tol->tol_corr, 1, st);
    st->steps++;
    if (ok) {
      t = t_new;
      for (int i = 0; i < n; ++i) x[i] = xp[i];
      if (++accepts == 3) {
        hstep = 2.0 * hstep < tol->h_max ? 2.0 * hstep : tol->h_max;
        accepts = 0;
      }
    } else {
      st->rejections++;
      hstep = 0.5 * hstep;
      accepts = 0;
    }
    if (norm_inf_dd(n, x) > tol->div_radius) { stat = REF_DIVERGED; break; }
    if (t >= 1.0) break;
    if (hstep < tol->h_min) { stat = REF_FAILED_MINSTEP; break; }
    if (st->steps > tol->max_steps) { stat = REF_FAILED_MAXSTEPS; break; }
  }
  cdd fx[MAXN];
  if (stat < 0) {
    /* t = 1: Newton on f in double-double, then the residual test */
    newton_dd(h, x, 1.0, tol->max_newton_final, tol->tol_final, 0, st);
    eval_f_ddj(h->f, x, fx, NULL);
    double res = norm_inf_dd(n, fx), nx = norm_inf_dd(n, x);
    st->residual = res;
    if (res <= tol->tol_residual && nx <= tol->div_radius) stat = REF_CONVERGED;
    else if (nx > tol->div_radius) stat = REF_DIVERGED;
    else stat = REF_FAILED_NEWTON_T1;
  } else {
    eval_f_ddj(h->f, x, fx, NULL);
    st->residual = norm_inf_dd(n, fx);
  }
  st->t_final = t;
  for (int i = 0; i < n; ++i) x_end[i] = x[i];
  *status = stat;
}

typedef struct {
  const homotopy *h;
  const double *start;
  const int64_t *ids;
  int64_t n_paths;
  const ref_tolerances *tol;
  double *ends_hi, *ends_lo;
  int32_t *status;
  ref_path_stats *stats;
  atomic_llong next;
} crew_dd;

static void *crew_dd_worker(void *arg) {
  crew_dd *c = (crew_dd *)arg;
  const int n = c->h->n;
  for (;;) {
    int64_t k = atomic_fetch_add(&c->next, 1);
    if (k >= c->n_paths) break;
    cplx xs[MAXN];
    if (c->start) {
      for (int i = 0; i < n; ++i) xs[i] = load(c->start + (size_t)2 * n * k, i);
    } else {
      double tmp[2 * MAXN];
      ref_start_point(n, c->h->deg, c->ids ? c->ids[k] : k, tmp);
      for (int i = 0; i < n; ++i) xs[i] = load(tmp, i);
    }
    cdd xe[MAXN];
    ref_path_stats st;
    int32_t s;
    track_one_dd(c->h, xs, c->tol, xe, &s, &st);
    for (int i = 0; i < n; ++i) {
      double *hi = c->ends_hi + (size_t)2 * n * k, *lo = c->ends_lo + (size_t)2 * n * k;
      hi[2 * i] = xe[i].re.hi;
      hi[2 * i + 1] = xe[i].im.hi;
      lo[2 * i] = xe[i].re.lo;
      lo[2 * i + 1] = xe[i].im.lo;
    }
    c->status[k] = s;
    if (c->stats) c->stats[k] = st;
  }
  return NULL;
}

int ref_track_paths_dd(const ref_system *f, const ref_system *g, const double *gamma,
                       const double *start, const int64_t *path_ids, int64_t n_paths,
                       const ref_tolerances *tol, double *ends_hi, double *ends_lo,
                       int32_t *status, ref_path_stats *stats, int32_t n_threads) {
  if (!f || f->n < 1 || f->n > MAXN || n_paths < 0 || !ends_hi || !ends_lo || !status) return -1;
  if (g && (g->n != f->n || !start)) return -1;
  ref_tolerances deftol;
  if (!tol) { ref_default_tolerances(&deftol); tol = &deftol; }
  homotopy h;
  if (make_homotopy(f, g, gamma, &h) != 0) return -1;
  crew_dd c;
  c.h = &h;
  c.start = start;
  c.ids = path_ids;
  c.n_paths = n_paths;
  c.tol = tol;
  c.ends_hi = ends_hi;
  c.ends_lo = ends_lo;
  c.status = status;
  c.stats = stats;
  atomic_init(&c.next, 0);
  if (n_threads < 1) n_threads = 1;
  if (n_threads == 1) {
    crew_dd_worker(&c);
    return 0;
  }
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -3;
  int started = 0;
  for (int i = 0; i < n_threads; ++i)
    if (pthread_create(&th[i], NULL, crew_dd_worker, &c) == 0) ++started;
  if (started == 0) crew_dd_worker(&c);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  return 0;
}
