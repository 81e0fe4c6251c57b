// Batched homotopy path tracker kernels for gfx950 (CDNA4), complex FP64.
//
// Work mapping.  A workgroup is W wavefronts; lane l of every wavefront
// belongs to the same path slot l, so a workgroup carries 64 paths.  Row r of
// the Jacobian (equation r) and component r of the path state live in wave
// r mod W, slot r / W.  Every wave streams the terms of its equations with
// wave-uniform (scalar) loads: the coefficient and the (variable, exponent)
// pairs of a term are the same for all 64 paths, so they sit in SGPRs and
// cost no vector bandwidth.  Per-path powers x_v^e are staged in LDS in a
// [v][e][lane] layout; reads use a wave-uniform offset and are lane
// contiguous.
//
// Method.  H(x,t) = gamma(1-t) g(x) + t f(x), g_i = x_i^{d_i} - 1 (paper:
// Section 1 and Section 2.2 for independent paths and dynamic load
// balancing).  f and its Jacobian are evaluated by reverse-mode algorithmic
// differentiation of each monomial (prefix products with the coefficient
// folded in, then a backward sweep of suffix products).  Linear systems are
// solved by Gauss-Jordan elimination with partial pivoting (largest
// |re|+|im| in the column, ties to the lowest row): the normalised pivot row
// is broadcast to the other waves through LDS.  One RK4 predictor step and
// up to max_newton Newton iterations form a step; the step control and the
// final Newton at t = 1 follow the library's documented reading.
//
// Scheduling.  The persistent kernel replaces the work crew's guarded
// next-job pointer (Section 1) with a device atomic queue head per system:
// after every step, lanes whose path finished claim new path ids with one
// atomicAdd per workgroup (ballot / popcount / mbcnt).  The plain kernel
// performs one step per launch for a fixed path -> lane map.
#include <hip/hip_runtime.h>

#include "hp_internal.hpp"

namespace hp {

struct cd {
  double re, im;
};

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// acc - a*b
__device__ __forceinline__ cd cfms(cd acc, cd a, cd b) {
  return {fma(-a.re, b.re, fma(a.im, b.im, acc.re)), fma(-a.re, b.im, fma(-a.im, b.re, acc.im))};
}
// 1/b by Smith's method
__device__ __forceinline__ cd crecip(cd b) {
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re;
    double id = 1.0 / (b.re + b.im * r);
    return {id, -r * id};
  }
  double r = b.re / b.im;
  double id = 1.0 / (b.re * r + b.im);
  return {r * id, -id};
}
__device__ __forceinline__ double cabs1(cd a) { return fabs(a.re) + fabs(a.im); }
__device__ __forceinline__ double cmod(cd a) { return sqrt(a.re * a.re + a.im * a.im); }
// max that propagates NaN from a (NaN never compares <=)
__device__ __forceinline__ double nmax(double m, double a) { return (a <= m) ? m : a; }

__device__ __forceinline__ cd ld(const double2 *p) {
  double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, cd v) { *p = make_double2(v.re, v.im); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

enum EvalMode { EV_NEG_HT = 0, EV_H = 1, EV_F = 2 };

template <int NMAX, int W>
struct Tracker {
  static constexpr int R = (NMAX + W - 1) / W;  // rows (and state components) per wave

  // ---- launch-wide ----
  const KArgs &a;
  const int lane, w;
  const int nl;  // LDS row stride: largest n of the launch
  // ---- LDS ----
  double2 *pw;    // [nl*emax][64] powers x_v^e, e = 1..emax
  double2 *jacc;  // [W][nl][64] Jacobian row accumulators (eval only)
  double2 *prow;  // [nl+1][64] normalised pivot row, [nl] = right-hand side
  double2 *dsol;  // [nl][64] solution of the last linear solve
  double *cand;   // [nl][64] pivot candidates
  double *red;    // [2W][64] cross-wave reductions
  long long *ctl; // [64] refill broadcast
  int *flag;      // [16] workgroup flags
  // ---- current system (wave-uniform) ----
  int n, emax, sysidx;
  const DevTerm *terms;
  const int32_t *eqp;
  cd gamma;
  const DevSys *sp;  // descriptor in global memory (scalar loads)
  long long npaths, out_path_base, out_x_base;
  const long long *ids;
  // ---- per-lane path state (replicated in every wave) ----
  int mode, accepts, steps, rejections, newton_its, evals, solves;
  long long qidx;  // queue index of the path in this slot
  double t, h;
  // ---- per-lane owned components ----
  cd x0[R], xc[R], ks[R];
  // ---- per-lane owned rows ----
  cd A[R][NMAX];
  cd b[R];

  __device__ Tracker(const KArgs &args, char *smem)
      : a(args), lane(threadIdx.x & 63), w(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)),
        nl(args.nl) {
    char *p = smem;
    pw = (double2 *)p;   p += sizeof(double2) * kLanes * nl * args.emax_all;
    // jacc (eval) and prow/dsol/cand (solve) share one region
    char *u = p;
    jacc = (double2 *)u;
    prow = (double2 *)u; u += sizeof(double2) * kLanes * (nl + 1);
    dsol = (double2 *)u; u += sizeof(double2) * kLanes * nl;
    cand = (double *)u;  u += sizeof(double) * kLanes * nl;
    p += lds_union_bytes(nl, W);
    red = (double *)p;   p += sizeof(double) * kLanes * 2 * W;
    ctl = (long long *)p; p += sizeof(long long) * kLanes;
    flag = (int *)p;
    mode = M_IDLE;
    t = 0.0;
    h = 0.0;
    qidx = 0;
    accepts = steps = rejections = newton_its = evals = solves = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) x0[i] = xc[i] = ks[i] = b[i] = {0.0, 0.0};
  }

  __device__ __forceinline__ void load_system(int s) {
    sysidx = s;
    sp = a.sys + s;
    n = sp->n;
    emax = sp->emax;
    terms = a.terms;
    eqp = a.eqp + sp->eq_base;
    gamma = {sp->gre, sp->gim};
    npaths = sp->n_paths;
    out_path_base = sp->out_path_base;
    out_x_base = sp->out_x_base;
    ids = (const long long *)sp->ids;
  }

  __device__ __forceinline__ int row_of(int i) const { return w + W * i; }

  // acc[v] += d for a wave-uniform v (scalar branches, no register indexing)
  __device__ __forceinline__ static void add_at(cd (&acc)[NMAX], int v, cd d) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j == v) acc[j] = cadd(acc[j], d);
  }

  // ------------------------------------------------------------------ eval
  // Terms with exactly K factors: value into f, partial derivatives added
  // into this wave's LDS accumulator row jac[v][lane] (ds_add_f64; each lane
  // owns its address).  Reverse-mode differentiation of the monomial:
  // prefix products P_m = c phi_0 ... phi_m, then a backward sweep with the
  // suffix product S, d/dx_{v_m} = P_{m-1} S e_m x_{v_m}^{e_m - 1}.
  template <int K>
  __device__ __forceinline__ void terms_k(int lo, int hi, cd &f, double2 *jac) {
#pragma nounroll
    for (int tt = lo; tt < hi; ++tt) {
      const DevTerm T = terms[tt];
      const cd c = {T.cre, T.cim};
      if constexpr (K == 0) {
        f = cadd(f, c);
      } else {
        int vv[K], ee[K];
        cd P[K];
        cd run = c;
#pragma unroll
        for (int m = 0; m < K; ++m) {
          const int byte = (T.w[(m + 1) >> 2] >> (8 * ((m + 1) & 3))) & 0xff;
          vv[m] = byte & 15;
          ee[m] = byte >> 4;
          run = cmul(run, ld(&pw[(vv[m] * emax + ee[m] - 1) * kLanes + lane]));
          P[m] = run;
        }
        f = cadd(f, run);
        cd S = {1.0, 0.0};
#pragma unroll
        for (int m = K - 1; m >= 0; --m) {
          const cd left = (m == 0) ? c : P[m > 0 ? m - 1 : 0];
          cd d = (m == K - 1) ? left : cmul(left, S);
          if (ee[m] > 1) {
            const cd q = ld(&pw[(vv[m] * emax + ee[m] - 2) * kLanes + lane]);
            d = cmul(d, cscale(q, (double)ee[m]));
          }
          double *acc = (double *)&jac[vv[m] * kLanes + lane];
          __hip_atomic_fetch_add(acc, d.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          __hip_atomic_fetch_add(acc + 1, d.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (m > 0) {
            const cd phi = ld(&pw[(vv[m] * emax + ee[m] - 1) * kLanes + lane]);
            S = (m == K - 1) ? phi : cmul(S, phi);
          }
        }
      }
    }
  }

  template <int K>
  __device__ __forceinline__ void terms_upto(const int32_t *kp, cd &f, double2 *jac) {
    if constexpr (K >= 0) {
      terms_upto<K - 1>(kp, f, jac);
      const int lo = kp[K], hi = kp[K + 1];
      if (lo < hi) terms_k<K>(lo, hi, f, jac);
    }
  }

  // Owned rows of J_x(xc, te) into A and, in b: -H_t (EV_NEG_HT), H (EV_H)
  // or f (EV_F) at (xc, te).
  __device__ __forceinline__ void eval(int emode, double te) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int j = row_of(i);
      if (j < n) {
        cd p = xc[i];
        st(&pw[(j * emax) * kLanes + lane], p);
        for (int e = 2; e <= emax; ++e) {
          p = cmul(p, xc[i]);
          st(&pw[(j * emax + e - 1) * kLanes + lane], p);
        }
      }
    }
    __syncthreads();
    double2 *jac = jacc + w * (nl * kLanes);
    const cd one = {1.0, 0.0};
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = row_of(i);
      if (r < n) {
#pragma nounroll
        for (int v = 0; v < n; ++v) jac[v * kLanes + lane] = make_double2(0.0, 0.0);
        cd f = {0.0, 0.0};
        terms_upto<NMAX>(eqp + r * kKSlots, f, jac);
        if (emode == EV_F) {
          b[i] = f;
          continue;
        }
        // start system g_r = x_r^{d_r} - 1
        const int d = sp->deg[r];
        cd xp = one;
        for (int e = 1; e < d; ++e) xp = cmul(xp, xc[i]);
        cd g = cmul(xp, xc[i]);
        g.re -= 1.0;
        const cd s = cscale(gamma, 1.0 - te);
        const cd sdg = cmul(s, cscale(xp, (double)d));
        if (emode == EV_H) {
          b[i] = cadd(cmul(s, g), cscale(f, te));
        } else {
          const cd ht = csub(f, cmul(gamma, g));
          b[i] = {-ht.re, -ht.im};
        }
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
          cd v = (j < n) ? ld(&jac[j * kLanes + lane]) : cd{0.0, 0.0};
          A[i][j] = cscale(v, te);
        }
        // diagonal of gamma (1-t) dg/dx: column r = w + W i, w in [0, W)
#pragma unroll
        for (int q = 0; q < W; ++q)
          if (q == w && i * W + q < NMAX) A[i][i * W + q] = cadd(A[i][i * W + q], sdg);
      }
    }
    __syncthreads();  // the accumulator rows alias the solver's LDS buffers
  }

  // ----------------------------------------------------------------- solve
  // Gauss-Jordan elimination with partial pivoting on the owned rows of
  // [A | b].  On return dsol[j] holds component j of the solution.  Returns
  // true for lanes whose matrix has an exactly zero (or NaN) pivot.
  __device__ __forceinline__ bool solve() {
    unsigned used = 0;
    int pc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) pc[i] = -1;
    bool sing = false;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k < n) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          int r = row_of(i);
          if (r < n) cand[r * kLanes + lane] = ((used >> i) & 1) ? -1.0 : cabs1(A[i][k]);
        }
        __syncthreads();
        double best = -1.0;
        int p = -1;
#pragma nounroll
        for (int r = 0; r < n; ++r) {
          double c = cand[r * kLanes + lane];
          if (c > best) {
            best = c;
            p = r;
          }
        }
        if (!(best > 0.0)) sing = true;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if (row_of(i) == p) {
            cd inv = crecip(A[i][k]);
#pragma unroll
            for (int j = 0; j < NMAX; ++j) {
              if (j > k && j < n) {
                A[i][j] = cmul(A[i][j], inv);
                st(&prow[j * kLanes + lane], A[i][j]);
              }
            }
            b[i] = cmul(b[i], inv);
            st(&prow[nl * kLanes + lane], b[i]);
            used |= 1u << i;
            pc[i] = k;
          }
        }
        __syncthreads();
        cd l[R];
        bool act[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          int r = row_of(i);
          act[i] = (r < n) && (r != p);
          l[i] = A[i][k];
        }
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
          if (j > k && j < n) {
            cd pj = ld(&prow[j * kLanes + lane]);
#pragma unroll
            for (int i = 0; i < R; ++i)
              if (act[i]) A[i][j] = cfms(A[i][j], l[i], pj);
          }
        }
        cd pb = ld(&prow[nl * kLanes + lane]);
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (act[i]) b[i] = cfms(b[i], l[i], pb);
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int r = row_of(i);
      if (r < n) {
        int c = (pc[i] >= 0 && pc[i] < n) ? pc[i] : r;
        st(&dsol[c * kLanes + lane], b[i]);
      }
    }
    __syncthreads();
    return sing;
  }

  // max over the workgroup's waves of (u, v) for this lane
  __device__ __forceinline__ void wg_max2(double &u, double &v) {
    red[(2 * w) * kLanes + lane] = u;
    red[(2 * w + 1) * kLanes + lane] = v;
    __syncthreads();
    double mu = 0.0, mv = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      mu = nmax(mu, red[(2 * q) * kLanes + lane]);
      mv = nmax(mv, red[(2 * q + 1) * kLanes + lane]);
    }
    __syncthreads();  // red may be rewritten right after
    u = mu;
    v = mv;
  }

  // ------------------------------------------------------------ start path
  __device__ __forceinline__ void start_path(long long q) {
    qidx = q;
    long long pid = ids ? ids[q] : q;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int j = row_of(i);
      if (j < n) {
        long long kk = (pid / sp->radix[j]) % sp->deg[j];
        double2 z = a.roots[sp->root_base + sp->root_off[j] + (int)kk];
        x0[i] = {z.x, z.y};
      }
    }
    mode = M_TRACK;
    t = 0.0;
    h = a.tol.h_init;
    accepts = steps = rejections = newton_its = evals = solves = 0;
  }

  // ------------------------------------------------------------- one step
  // One predictor-corrector attempt for TRACK lanes, the final Newton for
  // FINAL lanes.  Sets fin_status >= 0 for lanes whose path ends here (the
  // endpoint is then x0).  All control flow around barriers is uniform over
  // the workgroup because every wave holds identical per-lane state.  The
  // step runs as a sequence of phases that each make one evaluation (and one
  // solve), so eval() and solve() are instantiated once:
  //   0..3  RK4 stages (J k = -H_t), 4  Newton iterations (J dx = H),
  //   5     residual f(x0) of paths that end in this step.
  __device__ __forceinline__ void step(int &fin_status, double &fin_res) {
    const DevTol &tol = a.tol;
    const bool trk = (mode == M_TRACK);
    const bool fnl = (mode == M_FINAL);
    double hs = 0.0, tn = 1.0;
    if (trk) {
      if (h >= 1.0 - t) {
        hs = 1.0 - t;
        tn = 1.0;
      } else {
        hs = h;
        tn = t + h;
      }
    }
    const double th = t + 0.5 * hs;
    const int maxit = trk ? tol.max_newton : tol.max_newton_final;
    const double ntol = trk ? tol.tol_corr : tol.tol_final;
    bool ok = trk, iter = false, conv = false;
    int it = 0, fs = -1;
    double prev = 0.0, nx = 0.0, res = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) xc[i] = x0[i];
    int phase = ballot(trk) ? 0 : 4;
    if (phase == 4) iter = fnl;
    for (;;) {
      if (phase == 4 && ballot(iter) == 0) {
        // ---- step control ----
        if (trk) {
          ++steps;
          if (ok && conv) {
            t = tn;
#pragma unroll
            for (int i = 0; i < R; ++i) x0[i] = xc[i];
            if (++accepts == 3) {
              h = (2.0 * h < tol.h_max) ? 2.0 * h : tol.h_max;
              accepts = 0;
            }
          } else {
            ++rejections;
            h = 0.5 * h;
            accepts = 0;
          }
        }
        if (fnl) {
#pragma unroll
          for (int i = 0; i < R; ++i) x0[i] = xc[i];
        }
        double dummy = 0.0;
        nx = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (row_of(i) < n) nx = nmax(nx, cmod(x0[i]));
        wg_max2(nx, dummy);
        if (trk) {
          if (nx > tol.div_radius) fs = HP_DIVERGED;
          else if (t >= 1.0) mode = M_FINAL;
          else if (h < tol.h_min) fs = HP_FAILED_MINSTEP;
          else if (steps > tol.max_steps) fs = HP_FAILED_MAXSTEPS;
        }
        if (ballot(fs >= 0 || fnl) == 0) break;
        phase = 5;
#pragma unroll
        for (int i = 0; i < R; ++i) xc[i] = x0[i];
      }
      const double te = (phase == 0) ? (trk ? t : 1.0)
                      : (phase == 1 || phase == 2) ? (trk ? th : 1.0)
                      : (phase == 3 || phase == 4) ? tn : 1.0;
      eval(phase < 4 ? EV_NEG_HT : (phase == 4 ? EV_H : EV_F), te);
      if (phase == 5) {
        // ---- residual ||f(x0)||_inf of ending paths, classification ----
        double dummy = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (row_of(i) < n) res = nmax(res, cmod(b[i]));
        wg_max2(res, dummy);
        if (fnl) {
          if (res <= tol.tol_residual && nx <= tol.div_radius) fs = HP_CONVERGED;
          else if (nx > tol.div_radius) fs = HP_DIVERGED;
          else fs = HP_FAILED_NEWTON_T1;
        }
        break;
      }
      const bool sing = solve();
      if (phase < 4) {
        // ---- RK4 stage: k = dsol ----
        ok = ok && !sing;
        const double cnext = (phase == 2) ? hs : 0.5 * hs;
        const double wk = (phase == 0 || phase == 3) ? 1.0 : 2.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int j = row_of(i);
          const cd k = (j < n) ? ld(&dsol[j * kLanes + lane]) : cd{0.0, 0.0};
          ks[i] = (phase == 0) ? k : cadd(ks[i], cscale(k, wk));
          xc[i] = (phase == 3) ? cadd(x0[i], cscale(ks[i], hs / 6.0))
                               : cadd(x0[i], cscale(k, cnext));
        }
        if (phase == 3) {
          if (trk) {
            evals += 4;
            solves += 4;
          }
          if (fnl) {
#pragma unroll
            for (int i = 0; i < R; ++i) xc[i] = x0[i];
          }
          iter = (trk && ok) || fnl;
        }
        ++phase;
        continue;
      }
      // ---- Newton iteration: x -= dx ----
      double md = 0.0, mx = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int j = row_of(i);
        if (j < n) {
          const cd dx = ld(&dsol[j * kLanes + lane]);
          if (iter && !sing) xc[i] = csub(xc[i], dx);
          md = nmax(md, cmod(dx));
          mx = nmax(mx, cmod(xc[i]));
        }
      }
      wg_max2(md, mx);
      if (iter) {
        ++it;
        ++newton_its;
        ++evals;
        ++solves;
        const bool finite = (md < INFINITY) && (mx < INFINITY);
        if (sing || !finite) {
          iter = false;
        } else if (md <= ntol * (mx > 1.0 ? mx : 1.0)) {
          conv = true;
          iter = false;
        } else if (trk && it >= 2 && md > 0.5 * prev) {
          iter = false;
        } else {
          prev = md;
          if (it >= maxit) iter = false;
        }
      }
    }
    fin_status = fs;
    fin_res = res;
  }

  // Writes the finished path of this lane (queue index qidx of system sd).
  __device__ __forceinline__ void write_out(int fs, double res) {
    const long long o = out_path_base + qidx;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int j = row_of(i);
      if (j < n) a.endpoints[out_x_base + qidx * n + j] = make_double2(x0[i].re, x0[i].im);
    }
    if (w == 0) {
      a.status[o] = fs;
      if (a.stats) {
        hp_path_stats s;
        s.steps = steps;
        s.rejections = rejections;
        s.newton_iters = newton_its;
        s.evals = evals;
        s.solves = solves;
        s.pad = 0;
        s.t_final = t;
        s.residual = res;
        a.stats[o] = s;
      }
    }
  }
};

// ------------------------------------------------------------------------
// Persistent kernel: resident workgroups loop until every system's queue is
// drained.  A workgroup works on one system at a time and moves to the next
// system with work once its queue is empty and its own lanes are idle.
// ------------------------------------------------------------------------
template <int NMAX, int W>
__global__ void __launch_bounds__(64 * W) k_persistent(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Tracker<NMAX, W> tr(a, smem);
  int s = blockIdx.x % a.n_systems;
  int visited = 1;
  tr.load_system(s);
  bool exhausted = false;
  for (;;) {
    // ---- refill idle slots (wave 0 claims, all waves read) ----
    const bool idle = (tr.mode == M_IDLE);
    if (tr.w == 0) {
      const uint64_t m = ballot(idle);
      long long id = -1;
      int ex = exhausted ? 1 : 0;
      if (m != 0 && !exhausted) {
        const unsigned cnt = __popcll(m);
        unsigned long long base = 0;
        if (tr.lane == __builtin_ctzll(m))
          base = atomicAdd(&a.qhead[s], (unsigned long long)cnt);
        base = __shfl(base, __builtin_ctzll(m));
        const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        const long long q = (long long)base + rank;
        if (idle && q < tr.npaths) id = q;
        if ((long long)(base + cnt) >= tr.npaths) ex = 1;
      }
      tr.ctl[tr.lane] = id;
      if (tr.lane == 0) tr.flag[0] = ex;
    }
    __syncthreads();
    const long long q = tr.ctl[tr.lane];
    exhausted = tr.flag[0] != 0;
    __syncthreads();
    if (q >= 0) tr.start_path(q);
    if (ballot(tr.mode != M_IDLE) == 0) {
      if (!exhausted) continue;
      if (visited >= a.n_systems) break;
      s = (s + 1) % a.n_systems;
      ++visited;
      tr.load_system(s);
      exhausted = false;
      continue;
    }
    int fs;
    double res;
    tr.step(fs, res);
    if (fs >= 0) {
      tr.write_out(fs, res);
      tr.mode = M_IDLE;
    }
  }
}

// ------------------------------------------------------------------------
// Plain tracker: one step per launch.  Workgroup b owns queue indices
// [64 b, 64 b + 64) of the single system 0; state lives in HBM between steps.
// ------------------------------------------------------------------------
template <int NMAX>
__global__ void __launch_bounds__(64) k_plain_init(KArgs a) {
  const DevSys *sd = a.sys;
  const long long q = (long long)blockIdx.x * 64 + threadIdx.x;
  if (q >= sd->n_paths) return;
  const long long P = a.ps.P;
  const long long pid = sd->ids ? sd->ids[q] : q;
  for (int j = 0; j < sd->n; ++j) {
    long long kk = (pid / sd->radix[j]) % sd->deg[j];
    a.ps.x0[j * P + q] = a.roots[sd->root_base + sd->root_off[j] + (int)kk];
  }
  a.ps.t[q] = 0.0;
  a.ps.h[q] = a.tol.h_init;
  a.ps.iv[0 * P + q] = M_TRACK;
  for (int f = 1; f < 8; ++f) a.ps.iv[f * P + q] = 0;
}

template <int NMAX, int W>
__global__ void __launch_bounds__(64 * W) k_plain_step(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Tracker<NMAX, W> tr(a, smem);
  tr.load_system(0);
  const long long P = a.ps.P;
  const long long q = (long long)blockIdx.x * 64 + tr.lane;
  const bool valid = q < tr.npaths;
  int md = valid ? a.ps.iv[q] : (int)M_IDLE;
  if (ballot(md != M_IDLE) == 0) return;  // uniform over the workgroup
  tr.mode = md;
  tr.qidx = q;
  if (md != M_IDLE) {
    tr.t = a.ps.t[q];
    tr.h = a.ps.h[q];
    tr.accepts = a.ps.iv[1 * P + q];
    tr.steps = a.ps.iv[2 * P + q];
    tr.rejections = a.ps.iv[3 * P + q];
    tr.newton_its = a.ps.iv[4 * P + q];
    tr.evals = a.ps.iv[5 * P + q];
    tr.solves = a.ps.iv[6 * P + q];
#pragma unroll
    for (int i = 0; i < Tracker<NMAX, W>::R; ++i) {
      int j = tr.row_of(i);
      if (j < tr.n) {
        double2 z = a.ps.x0[j * P + q];
        tr.x0[i] = {z.x, z.y};
      }
    }
  }
  int fs;
  double res;
  tr.step(fs, res);
  if (fs >= 0) {
    tr.write_out(fs, res);
    tr.mode = M_IDLE;
  }
  if (md != M_IDLE) {
#pragma unroll
    for (int i = 0; i < Tracker<NMAX, W>::R; ++i) {
      int j = tr.row_of(i);
      if (j < tr.n) a.ps.x0[j * P + q] = make_double2(tr.x0[i].re, tr.x0[i].im);
    }
    if (tr.w == 0) {
      a.ps.t[q] = tr.t;
      a.ps.h[q] = tr.h;
      a.ps.iv[q] = tr.mode;
      a.ps.iv[1 * P + q] = tr.accepts;
      a.ps.iv[2 * P + q] = tr.steps;
      a.ps.iv[3 * P + q] = tr.rejections;
      a.ps.iv[4 * P + q] = tr.newton_its;
      a.ps.iv[5 * P + q] = tr.evals;
      a.ps.iv[6 * P + q] = tr.solves;
    }
  }
  if (tr.w == 0) {
    const uint64_t m = ballot(tr.mode != M_IDLE);
    if (tr.lane == 0 && m) atomicAdd(a.ps.active, (unsigned)__popcll(m));
  }
}

}  // namespace hp

// ------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------
using namespace hp;

// Dynamic LDS above the default per-workgroup limit must be opted into.
template <class K>
static int allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return (int)hipSuccess;
  return (int)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
}

template <int NMAX, int W>
static int launch_persistent_t(const KArgs &a, int groups, size_t lds, hipStream_t s) {
  int rc = allow_lds(k_persistent<NMAX, W>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_persistent<NMAX, W>), dim3(groups), dim3(64 * W), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, int W>
static int launch_plain_t(const KArgs &a, size_t lds, hipStream_t s) {
  int rc = allow_lds(k_plain_step<NMAX, W>, lds);
  if (rc) return rc;
  const int groups = (int)((a.ps.P + 63) / 64);
  hipLaunchKernelGGL((k_plain_step<NMAX, W>), dim3(groups), dim3(64 * W), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, int W>
static int occupancy_t(size_t lds, int *out) {
  int rc = allow_lds(k_persistent<NMAX, W>, lds);
  if (rc) return rc;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_persistent<NMAX, W>, 64 * W, lds);
}

// Compiled variants: one or two Jacobian rows per wave.
#define HP_DISPATCH(NM, WV, CALL)                          \
  switch (NM * 16 + WV) {                                   \
    case 4 * 16 + 2: return CALL(4, 2);                     \
    case 4 * 16 + 4: return CALL(4, 4);                     \
    case 8 * 16 + 4: return CALL(8, 4);                     \
    case 8 * 16 + 8: return CALL(8, 8);                     \
    case 12 * 16 + 6: return CALL(12, 6);                   \
    default: return (int)hipErrorInvalidValue;              \
  }

int hp_launch_persistent(int nmax, int waves, const KArgs &a, int groups, size_t lds, void *stream) {
#define CALLP(N, V) launch_persistent_t<N, V>(a, groups, lds, (hipStream_t)stream)
  HP_DISPATCH(nmax, waves, CALLP)
#undef CALLP
}

int hp_launch_plain_step(int nmax, int waves, const KArgs &a, size_t lds, void *stream) {
#define CALLS(N, V) launch_plain_t<N, V>(a, lds, (hipStream_t)stream)
  HP_DISPATCH(nmax, waves, CALLS)
#undef CALLS
}

int hp_max_groups_per_cu(int nmax, int waves, size_t lds, int *out) {
#define CALLO(N, V) occupancy_t<N, V>(lds, out)
  HP_DISPATCH(nmax, waves, CALLO)
#undef CALLO
}

int hp_launch_plain_init(int nmax, const KArgs &a, void *stream) {
  (void)nmax;
  const int groups = (int)((a.ps.P + 63) / 64);
  hipLaunchKernelGGL((k_plain_init<12>), dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
