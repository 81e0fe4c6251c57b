/*
 * homotopy.h -- C ABI of libhomotopy, a batched path tracker for polynomial
 * homotopies on AMD Instinct MI355X (gfx950), complex FP64 throughout.
 *
 * What it computes.  For a square polynomial system f(x) = 0 in n unknowns,
 * the library tracks the solution paths of
 *
 *     H(x, t) = gamma (1 - t) g(x) + t f(x),   t from 0 to 1,
 *
 * with the total-degree start system g_i(x) = x_i^{d_i} - 1 (d_i the degree
 * of f_i) and a random complex constant gamma.  The paths are independent of
 * each other, which makes the tracking embarrassingly parallel and lets
 * the work be handed out dynamically (paper: Section 1, the problem
 * statement and the work crew model; end of Section 2.1, tracking the paths
 * of a start system with dynamic load balancing; Section 3.2, Theorem 3.2 on
 * the speedup of tracking n paths with p workers).  Each endpoint comes back
 * classified, the finite / "at infinity" split of Section 3.1 (Figure 3).
 *
 * The tracking step itself is not given in the paper; the library follows
 * this reading: a fourth-order Runge-Kutta predictor on dx/dt = -J_x^{-1} H_t,
 * a Newton corrector at the new t (at most max_newton iterations, success
 * when ||dx||_inf <= tol_corr * max(1, ||x||_inf), failure when an iteration
 * does not halve the update), step halving on failure and doubling after
 * three successes (capped at h_max, last step clipped to t = 1), truncation
 * of paths with ||x||_inf > div_radius, and a final Newton at t = 1.  The
 * end game then refines the endpoint by Newton iterations with f evaluated
 * in double-double arithmetic (the paper's means to accuracy: Section 1,
 * Section 5.1), rounds it to the nearest double, and takes the residual test
 * ||f(x)||_inf <= tol_residual there with f again in double-double, so that
 * the endpoint and its classification do not depend on the order of the
 * double-precision arithmetic that led to it.
 *
 * Start points.  Path p (0 <= p < prod d_i) starts at x_i = exp(2 pi i k_i / d_i)
 * where p = sum_i k_i prod_{j<i} d_j (k_1 varies fastest).  Endpoint arrays
 * are indexed by path id.
 *
 * Conventions.
 *   - Return values: 0 on success or a negative HP_E_* code; the message of
 *     the last error on the calling thread is hp_last_error().
 *   - Ownership: the caller owns every buffer it passes.  Host inputs are
 *     copied before a call returns; the library never frees caller memory.
 *     A context owns its device workspace and stream.
 *   - Host arrays are plain host memory.  "_device" entry points take device
 *     pointers (e.g. from torch tensors) and run asynchronously on the given
 *     HIP stream (NULL: the context's stream).
 *   - Threads: one context per host thread.  A server is internally
 *     synchronised.
 */
#ifndef HOMOTOPY_H
#define HOMOTOPY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HP_MAX_N 12        /* largest number of unknowns */
#define HP_MAX_EXPONENT 15 /* largest exponent of one variable in a term */

/* error codes */
#define HP_OK 0
#define HP_E_INVALID_ARG (-1)
#define HP_E_UNSUPPORTED_N (-2)
#define HP_E_OOM (-3)
#define HP_E_DEVICE (-4)
#define HP_E_BUDGET (-5)

/* tracking modes */
#define HP_PLAIN 0   /* one kernel launch per step, host loop, static path map */
#define HP_BATCHED 1 /* one persistent launch, device atomic path-refill queue */

typedef struct { double re, im; } hp_c64;

/* A square system, CSR over equations.  Equation i owns the terms
 * eq_ptr[i] .. eq_ptr[i+1]-1; term k is coeff[k] * prod_j x_j^exps[k*n+j].
 * Requirements: 1 <= n <= HP_MAX_N, every exponent <= HP_MAX_EXPONENT, every
 * equation of degree >= 1 and at most HP_MAX_N variables per term. */
typedef struct {
  int32_t n;
  int32_t n_terms;
  const int32_t *eq_ptr; /* [n+1] */
  const hp_c64 *coeff;   /* [n_terms] */
  const uint8_t *exps;   /* [n_terms*n], dense exponent vectors */
} hp_system;

typedef struct {
  double tol_residual; /* 1e-10: CONVERGED needs ||f(x_end)||_inf <= this    */
  double tol_corr;     /* 1e-8:  Newton corrector relative update size        */
  double tol_final;    /* 1e-13: final Newton at t = 1, relative update size  */
  double div_radius;   /* 1e8:   ||x||_inf beyond this -> DIVERGED (truncate)  */
  double h_init;       /* 0.01 */
  double h_min;        /* 1e-13: smaller step -> FAILED_MINSTEP               */
  double h_max;        /* 0.1 */
  int32_t max_steps;        /* 10000: more attempts -> FAILED_MAXSTEPS */
  int32_t max_newton;       /* 3 */
  int32_t max_newton_final; /* 6 */
} hp_tolerances;

typedef enum {
  HP_CONVERGED = 0,        /* finite endpoint, residual test passed          */
  HP_DIVERGED = 1,         /* ||x||_inf > div_radius ("at infinity")         */
  HP_FAILED_MINSTEP = 2,   /* step size fell below h_min before t = 1        */
  HP_FAILED_MAXSTEPS = 3,  /* more than max_steps attempts                   */
  HP_FAILED_NEWTON_T1 = 4  /* reached t = 1 but the residual test failed     */
} hp_status;

typedef struct {
  int32_t steps;        /* predictor-corrector attempts                       */
  int32_t rejections;   /* rejected attempts                                  */
  int32_t newton_iters; /* corrector iterations, final Newton included        */
  int32_t evals;        /* evaluations of H and J_x (predictor + corrector)   */
  int32_t solves;       /* linear solves                                      */
  int32_t pad;
  double t_final;       /* t where tracking stopped                           */
  double residual;      /* ||f(x_end)||_inf (double-double f for paths that  */
                        /* reached t = 1 with a finite endpoint)              */
} hp_path_stats;

typedef struct {
  double kernel_ms;   /* device time of the tracking kernels (HIP events)     */
  double endgame_ms;  /* device time of the end game after them (HIP events)  */
  double post_ms;     /* host wall time of a solve's duplicate post-pass      */
  double total_ms;    /* host wall time of the whole call                     */
  int64_t launches;   /* tracking kernel launches                             */
  int32_t paths_per_wave; /* paths one wavefront holds at a time          */
  int32_t max_n;      /* compiled size bound n_max of the variant used        */
  int32_t groups;     /* workgroups (one wavefront each) launched             */
  int32_t variant;    /* kernel variant code (see hp_plan_set_variant)        */
  int32_t lanes_per_path; /* 1 (one path per lane) or n (group kernels)      */
  int32_t waves_per_simd; /* cap on resident wavefronts per SIMD (0: none)   */
} hp_timing;

/* A launch configuration chosen by the autotuner (hp_plan_tuning,
 * hp_tune_batch): the kernel variant (which fixes the lanes per path),
 * paths per wavefront and the cap on resident wavefronts per SIMD, with the
 * kernel time of the choice and of the untuned default on the sample. */
typedef struct {
  int32_t variant;
  int32_t lanes_per_path;
  int32_t paths_per_wave;
  int32_t waves_per_simd; /* 0: as many as fit                               */
  double ms;              /* sample kernel time of the choice (0 if cached)  */
  double ms_default;      /* sample kernel time of the default shape         */
  int32_t candidates;     /* configurations timed                           */
  int32_t cached;         /* 1: taken from the tuning cache, nothing timed   */
} hp_tune_choice;

typedef struct hp_context hp_context;
typedef struct hp_plan hp_plan;
typedef struct hp_server hp_server;

/* Context on HIP device `device`.  Creates a stream of default priority.
 * A call that takes a context, a plan or a server may make the context's
 * device the current HIP device of the calling thread, and leaves it so. */
int hp_context_create(int device, hp_context **out);
/* Ends the caller's use of ctx.  Plans and servers made from ctx may be
 * destroyed before or after it: the context's stream and events are
 * released once ctx and all of them are destroyed, so no order of
 * destruction leaves a plan or server with a freed context (they stay
 * usable until destroyed). */
void hp_context_destroy(hp_context *ctx);
/* Message of the last failed call on this thread ("" if none). */
const char *hp_last_error(void);
void hp_default_tolerances(hp_tolerances *tol);
/* Timing of the last tracking call made with ctx. */
int hp_last_timing(const hp_context *ctx, hp_timing *out);
/* Number of total-degree paths of f (prod of equation degrees); -1 if invalid
 * or larger than 2^62. */
int64_t hp_path_count(const hp_system *f);

/* Host-memory call, the problem statement's track_paths(system,
 * start_solutions, gamma, tolerances): tracks n_paths paths of
 * gamma (1 - t) g + t f from t = 0 to t = 1.
 *   g == NULL, start == NULL: total-degree start system, paths 0..n_paths-1
 *     with their start points decoded from the path ids (see above);
 *   g == NULL, start != NULL: total-degree start system, path k starts at
 *     start[k*n .. k*n+n-1] (any solutions of x_i^{d_i} = 1);
 *   g != NULL, start != NULL: a general start system of the same n (its
 *     own terms, e.g. f with other coefficients: coefficient-parameter
 *     continuation), path k starting at start[k*n ..] (solutions of g);
 *   g != NULL, start == NULL: HP_E_INVALID_ARG.
 *   endpoints [n_paths*n], status [n_paths], stats [n_paths] or NULL.
 *   mode: HP_PLAIN or HP_BATCHED.  General start systems and explicit
 *   start points run on the group kernels. */
int hp_track_paths(hp_context *ctx, const hp_system *f, const hp_system *g, const hp_c64 *start,
                   int64_t n_paths, hp_c64 gamma, const hp_tolerances *tol, hp_c64 *endpoints,
                   int32_t *status, hp_path_stats *stats, int32_t mode);

/* The double-double tracker (the paper's "quality up": Section 1; Section
 * 5.1 and Table 2 run the solver in double-double): the homotopy, predictor,
 * corrector, step control and end game of hp_track_paths with every
 * operation on points, values, Jacobians and linear systems in complex
 * double-double (t and h in double), the final Newton at t = 1 in
 * double-double to tol->tol_final and the residual ||f(x)||_inf with f in
 * double-double.  Total-degree start system; start == NULL: paths
 * 0..n_paths-1 decoded from their ids, else path k starts at start[k*n..].
 * Endpoints as double-double pairs: endpoints_hi + endpoints_lo, each
 * [n_paths*n]; status [n_paths], stats [n_paths] or NULL.  Host memory.
 * One path per group of n lanes on the device. */
int hp_track_paths_dd(hp_context *ctx, const hp_system *f, const hp_c64 *start, int64_t n_paths,
                      hp_c64 gamma, const hp_tolerances *tol, hp_c64 *endpoints_hi,
                      hp_c64 *endpoints_lo, int32_t *status, hp_path_stats *stats);
/* The double-double tracker's defaults: hp_default_tolerances with the final
 * Newton run to tol_final = 1e-26. */
void hp_default_tolerances_dd(hp_tolerances *tol);

/* A plan: f packed and resident on the device, with a kernel variant chosen
 * (autotuned when tune != 0 and no cached choice exists).  Without tuning,
 * a plan for n <= 10 whose terms have at most 1024 factors in all runs on a
 * kernel specialised to f's support (variant 300 + n): its source is written
 * and compiled (hiprtc) at plan creation, which takes seconds (n = 8: 5-7 s,
 * n = 10: 13-17 s on one host core) the first time a support is seen; plans
 * for systems of the same support share the compiled module, and
 * $HP_JIT_CACHE (a directory) keeps code objects across processes (keyed by
 * the source, the compiler version and options and the library's kernel
 * headers, so a rebuilt library does not load stale code).  Errors of that
 * compilation are HP_E_DEVICE with the compiler log in hp_last_error. */
int hp_plan_create(hp_context *ctx, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
                   int32_t tune, hp_plan **out);
/* A plan for gamma (1 - t) g + t f with explicit start points (host array
 * [n_start][n], copied; path id k starts at row k; g as for hp_track_paths,
 * NULL for the total-degree start system).  When g has f's support term by
 * term (the same equations with the same monomials in the same order, other
 * coefficients: the coefficient-parameter continuation of Section 2.1, the
 * "contin" stage of Section 5.4 Table 5) and n <= 10, the default variant is
 * the specialised kernel in its coefficient-parameter form: one sweep over
 * the monomials with the blended coefficients gamma (1 - t) cg + t cf gives
 * J and H, and the coefficients gamma cg - cf give -H_t.  Otherwise, and for
 * every other g, the group kernels.  tune != 0 runs the autotuner as for
 * hp_plan_create.  HP_E_INVALID_ARG for a missing start array or a g of
 * another n. */
int hp_plan_create_general(hp_context *ctx, const hp_system *f, const hp_system *g,
                           const hp_c64 *start, int64_t n_start, hp_c64 gamma,
                           const hp_tolerances *tol, int32_t tune, hp_plan **out);
void hp_plan_destroy(hp_plan *plan);
/* Forces the kernel variant.  Three kernel families:
 *   n_max = 4, 8, 10, 12   group kernels: n lanes of a wavefront per path
 *                          (lane r owns equation r), floor(64/n) paths, for
 *                          any n <= n_max;
 *   100 + n (n = 1..8)     lane kernels: one path per lane, 64 paths per
 *                          wavefront, Jacobian in LDS, compiled for exactly
 *                          this n;
 *   200 + n (n = 7, 8)     lane kernels with 32 paths per wavefront (half the
 *                          LDS, for systems whose power table is large);
 *   300 + n (n = 1..10)    the kernel specialised to the plan's system (one
 *                          path per lane, [J | rhs] in registers, compiled at
 *                          run time; total-degree start system, or a start
 *                          system on f's support: hp_plan_create_general);
 *   400, 411, 412          dense kernels for equations of total degree <= 3
 *                          (400: any n <= 10; 411, 412: n = 11, 12), one path
 *                          per lane, batched mode only (a plain call of a
 *                          plan on a dense kernel runs a group kernel).
 * The variant must fit the system's n and its LDS must fit the device; 0
 * selects the default (the specialised kernel where it applies, else a
 * dense kernel for a dense system of total degree <= 3, else the narrowest
 * group kernel).  HP_E_INVALID_ARG for other values,
 * HP_E_UNSUPPORTED_N if the LDS does not fit.  The autotuner of
 * hp_plan_create times every candidate on a sample of the plan's paths and
 * caches the choice per system shape (file named by $HP_TUNE_CACHE). */
int hp_plan_set_variant(hp_plan *plan, int32_t variant);
/* Launch shape of the plan's variant: paths_per_wave (1..64; 0: all 64) for
 * the specialised and dense kernels (other variants take 0 only), and a cap
 * on the resident wavefronts per SIMD (0: as many as fit).  Paths are
 * tracked independently (Section 1), so a path's result does not depend on
 * the shape.  HP_E_INVALID_ARG for values out of range. */
int hp_plan_set_launch(hp_plan *plan, int32_t paths_per_wave, int32_t waves_per_simd);
/* The autotuner's record for a plan created with tune != 0 (zeros
 * otherwise).  The tuner times every compiled variant that fits the
 * system (group kernels: n lanes per path; lane, specialised and dense
 * kernels: one), for the specialised and dense kernels with 64 and 32 paths
 * per wavefront, each with every binding cap on the wavefronts per SIMD, on
 * a sample of the plan's paths (2 resident rounds), and caches the fastest
 * by device and system shape (n, terms, largest exponent and factor count)
 * in memory and in the file $HP_TUNE_CACHE names. */
int hp_plan_tuning(const hp_plan *plan, hp_tune_choice *out);

/* Writes and compiles the kernel specialised to f (variant 300 + n) for
 * gfx950 without loading it, so it needs no device, in its two forms: the
 * plans' and the server's (which suspends and resumes paths);
 * *code_bytes = size of the plans' code object.  The code objects are kept
 * for the process (and written to the directory $HP_JIT_CACHE names, when
 * set, where later processes find them), so plans and servers for systems
 * with f's support skip the compilation: a caller can compile ahead of the
 * first solve.  HP_E_UNSUPPORTED_N when f cannot have one (n > 10, or more
 * than 1024 factors in all), HP_E_DEVICE when compilation fails (compiler log
 * in hp_last_error), HP_E_INVALID_ARG for a malformed system. */
int hp_spec_compile(const hp_system *f, int64_t *code_bytes);
/* One form of that kernel: 0 the plans', 1 the server's, 2 the
 * coefficient-parameter form of hp_plan_create_general (which depends on
 * f's support only).  Same errors; HP_E_INVALID_ARG for another form. */
int hp_spec_compile_form(const hp_system *f, int32_t form, int64_t *code_bytes);

/* Device-memory call: tracks the paths whose ids are ids[0..n_paths-1]
 * (device int64 array; NULL means ids 0..n_paths-1).  Outputs are device
 * arrays indexed like ids: endpoints [n_paths*n] hp_c64, status [n_paths],
 * stats [n_paths] or NULL.  Asynchronous on `stream` (NULL: context stream)
 * except in HP_PLAIN mode, whose host step loop reads an active-path count
 * back after every launch.  Ids must be < hp_path_count. */
int hp_plan_track_device(hp_plan *plan, const int64_t *ids, int64_t n_paths, hp_c64 *endpoints,
                         int32_t *status, hp_path_stats *stats, int32_t mode, void *stream);

/* Many systems of different n in one persistent launch (one refill queue per
 * system), the batched form of the work crew: the paper's speedup of
 * tracking n paths with p workers is bounded by the tail of n mod p paths
 * (Section 3.2, Theorem 3.2) and, for a sequence of path sets, by one tail
 * per set (the corollary after it); one launch over all systems leaves one
 * tail for the whole batch instead of one per system.  System s owns the paths path_offsets[s] .. path_offsets[s+1]-1
 * of the output (path_offsets[0] = 0, path_offsets[s+1] - path_offsets[s] =
 * hp_path_count(&fs[s])); its endpoints start at hp_c64 index x_offsets[s]
 * (x_offsets[s+1] = x_offsets[s] + paths_s * n_s).  Both offset arrays have
 * n_systems+1 entries and are written by hp_batch_layout.  Host memory. */
int hp_batch_layout(const hp_system *fs, int32_t n_systems, int64_t *path_offsets,
                    int64_t *x_offsets);
int hp_track_batch(hp_context *ctx, const hp_system *fs, int32_t n_systems,
                   const hp_c64 *gammas, const hp_tolerances *tol, hp_c64 *endpoints,
                   int32_t *status, hp_path_stats *stats);
/* Autotunes the launch of a batch (the variants that run every system of
 * it: the dense kernels, the group kernels; the launch shapes as for
 * hp_plan_tuning) on a sample of each system's paths and caches the
 * choice by device and batch shape (number of systems, range of n, terms,
 * largest exponent and factor count, dense or not); hp_track_batch calls on
 * batches of that shape launch with it.  Arguments as for hp_track_batch. */
int hp_tune_batch(hp_context *ctx, const hp_system *fs, int32_t n_systems, const hp_c64 *gammas,
                  const hp_tolerances *tol, hp_tune_choice *out);

/* Endpoint post-pass (host): pairs (a, b), a < b, of CONVERGED endpoints with
 * ||x_a - x_b||_inf <= rel * max(1, ||x_a||_inf), found by sorting on a random
 * real projection and comparing within a window.  Writes up to max_pairs
 * pairs to pairs[2k], pairs[2k+1]; returns the number of pairs found. */
int64_t hp_find_duplicates(int32_t n, int64_t n_paths, const hp_c64 *endpoints,
                           const int32_t *status, double rel, int64_t *pairs, int64_t max_pairs);

/* Device-memory duplicate scan, the same pairs as hp_find_duplicates (any
 * order): endpoints [n_paths*n] and status [n_paths] are device arrays (as
 * hp_plan_track_device writes them); up to max_pairs pairs go to the device
 * array pairs[2*max_pairs] (NULL if max_pairs is 0); *n_pairs (host) receives
 * the number of pairs found, which may exceed max_pairs.  The converged
 * endpoints are projected and sorted on the device (workspace owned by ctx,
 * grown on demand); the call waits for `stream` (NULL: the context's) to
 * read two counts back. */
int hp_find_duplicates_device(hp_context *ctx, int32_t n, int64_t n_paths, const hp_c64 *endpoints,
                              const int32_t *status, double rel, int64_t *pairs, int64_t max_pairs,
                              int64_t *n_pairs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the scan of
 * hp_find_duplicates_device, same arguments and results, in a workspace the
 * library holds per GPU for the life of the process (a fixed array of about
 * 36 MiB on each GPU it runs on) instead of memory it allocates; the call
 * allocates nothing.  At most 524,288 converged endpoints per call
 * (HP_E_BUDGET beyond).  Every call on a GPU uses that GPU's one workspace:
 * calls that overlap on one GPU race, so callers serialise them. */
int hp_find_duplicates_device_static(hp_context *ctx, int32_t n, int64_t n_paths,
                                     const hp_c64 *endpoints, const int32_t *status, double rel,
                                     int64_t *pairs, int64_t max_pairs, int64_t *n_pairs,
                                     void *stream);

/* The solve of the plan's system with device outputs: every total-degree
 * path (HP_BATCHED, end game included) into endpoints [P*n], status [P] and
 * stats [P] (nullable), P = hp_path_count; then the duplicate post-pass of
 * hp_solve on the device: pairs at 1e-6 relative (*pairs_found), both paths
 * of each tracked once more with h_max = min(h_max, 0.01) and tol_corr =
 * min(tol_corr, 1e-10) and written back in place, and the pairs left
 * counted (*pairs_left; both host pointers, nullable).  Returns when the
 * outputs are complete on `stream` (NULL: the context's). */
int hp_plan_solve_device(hp_plan *plan, hp_c64 *endpoints, int32_t *status, hp_path_stats *stats,
                         int64_t *pairs_found, int64_t *pairs_left, void *stream);

/* Tracks all paths of f (HP_BATCHED), then re-tracks both paths of every
 * duplicate pair once with h_max = min(h_max, 0.01) and tol_corr =
 * min(tol_corr, 1e-10).  *remaining_pairs receives the duplicate pairs left
 * afterwards.  Host memory, like hp_track_paths. */
int hp_solve(hp_context *ctx, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
             hp_c64 *endpoints, int32_t *status, hp_path_stats *stats, int64_t *remaining_pairs);

/* Homotopy membership test (Section 4.1, Example 4.1): whether test points
 * lie on a positive-dimensional solution set given by witness points.
 *   e: the embedded system (Section 2.1): its last n_hyper equations are the
 *      linear hyperplanes that cut the set (degree 1; each may have a
 *      constant term);
 *   witness [m*n]: the m witness points (solutions of e on the set);
 *   tests [n_tests*n]: points to test, in e's unknowns (slack variables 0).
 * For each test point y the witness points are tracked along
 * (1 - t) e + t e_y, where e_y is e with the constant of each hyperplane
 * replaced so that it passes through y (gamma = 1: only those constants
 * move, c0 to c3); all tests run in one persistent launch.  Outputs (host):
 * endpoints [n_tests*m*n], status [n_tests*m], member [n_tests] = 1 when a
 * CONVERGED endpoint of that test satisfies ||x - y||_inf <= rel max(1,
 * ||y||_inf).  HP_E_INVALID_ARG if a hyperplane equation is not linear. */
int hp_membership_test(hp_context *ctx, const hp_system *e, int32_t n_hyper, const hp_c64 *witness,
                       int64_t m, const hp_c64 *tests, int32_t n_tests, const hp_tolerances *tol,
                       double rel, hp_c64 *endpoints, int32_t *status, int32_t *member);

/* Cascade of homotopies (Section 3.1, Example 3.1, Figure 3): candidate
 * generic points on the solution sets of every dimension k, k-1, .., 0.
 *   e: an embedded system (Section 2.1) of top dimension k: unknowns
 *      (x_1..x_{n-k}, z_1..z_k), equations f_i + sum_j gamma_ij z_j
 *      (i < n - k), then the k hyperplanes, hyperplane j holding z_j;
 *   gammas [k+1]: the random constant of each stage's homotopy.
 * Stage 0 solves e (hp_plan_solve_device: every total-degree path, end
 * game, duplicate post-pass); its CONVERGED endpoints with |z_k| <=
 * slack_tol are the candidates of dimension k, those with z_k != 0 the start
 * points of stage 1.  Stage s (dimension d = k - s) tracks them with
 * gammas[s] from the previous system to the one where z_{d+1} leaves the
 * first n - k equations and its hyperplane becomes z_{d+1} = 0 (a general
 * start system, so the group kernels); its CONVERGED endpoints with
 * |z_d| <= slack_tol are the candidates of dimension d, the rest start
 * stage s + 1; at dimension 0 every CONVERGED endpoint is a candidate.
 * Outputs (host): stages [k+1]; the first min(total, cap) candidates in
 * witness [cap*n] with their dimensions in witness_dim [cap], stage after
 * stage; *n_witness = total candidates. */
typedef struct {
  int32_t dim;            /* dimension of the stage's candidates           */
  int32_t pad;
  int64_t paths;          /* paths tracked in the stage                    */
  int64_t converged;
  int64_t candidates;     /* converged with zero slack (dim 0: converged)  */
  int64_t nonzero;        /* converged with nonzero slack: next stage      */
  double kernel_ms;       /* tracking kernel time of the stage             */
} hp_cascade_stage;
int hp_cascade(hp_context *ctx, const hp_system *e, int32_t k, const hp_c64 *gammas,
               const hp_tolerances *tol, double slack_tol, hp_cascade_stage *stages,
               hp_c64 *witness, int32_t *witness_dim, int64_t cap, int64_t *n_witness);

/* Serving: a request loop with continuous batching (a worker thread with its
 * own stream), in the manner of the paper's pipeline in which tracking of
 * the paths of one piece of work starts while other pieces are still being
 * produced (Section 2.2, Figure 1: a producer stage feeding tracking
 * threads), with the paths tracked independently of one another (Section 1),
 * which is what lets a path stop and resume between launches.  The server
 * allocates an arena of at most hbm_budget_bytes: path slots of HP_MAX_N
 * endpoint coordinates + status + stats (236 B each).  Requests (one system
 * each, all its total-degree paths) are admitted in arrival order while
 * their slot regions fit (at most 262,144 slots each; a request with more
 * paths, or one larger than the free room, which gets at least 4096 slots,
 * reuses the slots of its finished paths).
 * The work goes in epochs.  Each epoch packs a queue of paths of the
 * admitted requests (same tolerances), in admission order up to 524,288
 * paths, into one multi-system persistent launch per kernel family (the
 * kernel specialised to a support, shared by the requests of that support;
 * the dense kernels; the group kernels), so that requests that arrive while
 * others run share the following launches, the oldest requests finish
 * first under load, and each request runs on the kernel it would get alone.
 * On the specialised and dense kernels each wavefront stops after a budget
 * of steps per epoch: its paths in flight are suspended in their slots (the
 * accepted point, t, the step size and the counters) and resume from there
 * in a later epoch, bit for bit as if never stopped.  The budget of each
 * family adapts so that its epoch's kernel time is about the slice time
 * (hp_server_set_slice), which bounds how long a new request waits before
 * its paths start when the epochs have room for them.  The group kernels
 * run their queue to the end.
 * HP_E_BUDGET if the budget holds fewer than 4096 slots. */
int hp_server_create(hp_context *ctx, size_t hbm_budget_bytes, hp_server **out);
/* Time slicing of the specialised and dense kernel families: slice_ms is the
 * target kernel time of an epoch (default 50 ms), fixed_steps > 0 replaces
 * the adaptive budget by that many steps per wavefront and epoch, and
 * slice_ms = fixed_steps = 0 runs every queue to the end.  Results do not
 * depend on these settings.  Takes effect from the next epoch; HP_E_INVALID_ARG
 * for a negative or non-finite value. */
int hp_server_set_slice(hp_server *srv, double slice_ms, int32_t fixed_steps);
typedef struct hp_server_info {
  int64_t epochs;        /* epochs run so far                                */
  int64_t carried;       /* queue entries left unfinished at the end of an
                            epoch (suspended or not started), summed          */
  double epoch_ms_max;   /* longest epoch, wall time from queue build to the
                            end of the harvest                               */
  double epoch_ms_mean;
  double slice_ms;       /* settings of hp_server_set_slice                  */
  int32_t fixed_steps;
  int32_t budget_min;    /* smallest and largest adaptive step budget of the
                            families seen (0: none yet)                      */
  int32_t budget_max;
  int32_t pad;
  uint64_t peak_bytes;   /* as hp_server_peak_bytes                          */
} hp_server_info;
int hp_server_info_get(hp_server *srv, hp_server_info *out);
/* Queues a request; the system is copied.  *req_id receives its id.  A
 * sparse system with n <= 10 runs on the kernel specialised to its support;
 * the first time that support is seen in the process the server compiles it
 * (seconds) on its compile thread, not in this call, and the request waits
 * for it; the calling thread's current HIP device becomes the server's. */
int hp_server_submit(hp_server *srv, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
                     int64_t *req_id);
/* *done = 1 once every path of the request has finished (non-blocking). */
int hp_server_poll(hp_server *srv, int64_t req_id, int32_t *done);
/* Blocks until the request is done, then copies its results (host arrays
 * sized for hp_path_count paths; stats may be NULL) and forgets it.
 * *latency_ms (nullable) receives completion time minus submission time. */
int hp_server_wait(hp_server *srv, int64_t req_id, hp_c64 *endpoints, int32_t *status,
                   hp_path_stats *stats, double *latency_ms);
/* Peak bytes of arena slots held by admitted requests so far (<= budget). */
int hp_server_peak_bytes(hp_server *srv, size_t *out);
/* Stops the worker and the compile thread; requests not yet finished end as
 * failed.  No other thread may be inside a call on srv (hp_server_wait
 * included) while it runs. */
void hp_server_destroy(hp_server *srv);

#ifdef __cplusplus
}
#endif
#endif
