// The double-double tracker for gfx950: the paper's "quality up" (Section 1;
// Section 5.1 and Table 2 run the blackbox solver in double-double) on the
// device.  The same homotopy, RK4 predictor, Newton corrector, step control
// and end game as the double-precision tracker, with every operation on
// points, function values, Jacobians and linear systems in complex
// double-double; t and h stay doubles.  The final Newton at t = 1 runs in
// double-double to tol_final and the residual is ||f(x)||_inf with f in
// double-double.
//
// Mapping.  A path is a group of N consecutive lanes (N = n, one
// instantiation per n = 1..12): lane r owns equation r, row r of [J | rhs]
// and unknown r of the path's state, so a lane holds N + 1 complex
// double-double entries of the Jacobian, not N (N + 1), and every n up to
// 12 fits the registers; floor(64 / N) paths per wavefront.  Lane r
// evaluates equation r from the equation-ordered term table (coefficient and
// a dense exponent vector of 4 bits per variable, so variable indices are
// compile-time constants), with the whole point broadcast through LDS.  The
// linear solve is Gauss-Jordan elimination across the group's lanes with
// partial pivoting (largest |re| + |im| of the nearest double in the column,
// ties to the lowest row: the pivots of the oracle's LU), the pivot row
// exchanged and broadcast through LDS.  A group claims its next path from
// the system's device queue head with one atomic when its path is done.
#include <hip/hip_runtime.h>

#include "hp_device.hpp"
#include "hp_internal.hpp"
#include "lane_track.hpp"  // cptr, as_const

#include "dd_arith.hpp"  // switches floating-point contraction off for this file

namespace hp {
namespace {

// LDS of one path group
template <int N>
struct DdGroup {
  cdd x[N];         // the point, broadcast
  cdd prow[N + 1];  // normalised pivot row (or the row moving to the pivot's place)
  cdd srow[N + 1];  // the row moving from the pivot's place
  double cand[N];   // pivot candidates
  double red[N];    // reductions
  long long q;      // path claimed by the group
};

template <int N>
struct DdTrack {
  static constexpr int kGroups = kLanes / N;
  const KArgs &a;
  DdGroup<N> *G;
  const int lane, grp, r;
  const bool slot;  // the lane belongs to a path group
  cptr<DevSys> sp;
  cd gamma;
  int deg_r;
  cptr<double> coef;
  cptr<uint32_t> ex;
  int t0, t1;  // this lane's equation: terms t0 .. t1-1
  // group state (the same in every lane of the group)
  int mode, accepts, steps, rejections, newton_its, evals, solves;
  long long qidx;
  double t, h;
  // own component and row
  cdd x0, ks, xc;
  cdd A[N];
  cdd b;

  __device__ DdTrack(const KArgs &args, DdGroup<N> *groups)
      : a(args), lane(threadIdx.x & 63), grp((threadIdx.x & 63) / N),
        r((threadIdx.x & 63) - ((threadIdx.x & 63) / N) * N), slot(grp < kGroups) {
    G = groups + grp;  // lanes past the last group use the spare group
    sp = as_const(a.sys);
    gamma = {sp->gre, sp->gim};
    const int rr = slot ? r : 0;
    deg_r = sp->deg[rr];
    coef = as_const((const double *)a.tcoef) + 2 * (long long)sp->eg_base;
    ex = as_const((const uint32_t *)a.tmeta) + 4 * (long long)sp->eg_base;
    t0 = sp->eg_ptr[rr];
    t1 = sp->eg_ptr[rr + 1];
    mode = M_IDLE;
    accepts = steps = rejections = newton_its = evals = solves = 0;
    qidx = 0;
    t = h = 0.0;
    x0 = ks = xc = b = cdd_zero();
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] = cdd_zero();
  }

  // max over the group's lanes
  __device__ __forceinline__ double group_max(double v) {
    G->red[r] = v;
    wsync();
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) m = nmax(m, G->red[j]);
    wsync();
    return m;
  }

  // start point of path q: digit r of the id in the mixed radix of the
  // degrees picks the root of unity of x_r
  __device__ __forceinline__ void start_path(long long q) {
    qidx = q;
    const long long pid = sp->ids ? ((const long long *)sp->ids)[q] : sp->id_base + q;
    if (sp->start) {
      const double2 z = sp->start[pid * N + r];
      x0 = to_cdd({z.x, z.y});
    } else {
      cptr<double> roots = as_const((const double *)a.roots) + 2 * sp->root_base;
      const long long kk = (pid / sp->radix[r]) % deg_r;
      const int ri = sp->root_off[r] + (int)kk;
      x0 = to_cdd({roots[2 * ri], roots[2 * ri + 1]});
    }
    ks = cdd_zero();
    mode = M_TRACK;
    t = 0.0;
    h = a.tol.h_init;
    accepts = steps = rejections = newton_its = evals = solves = 0;
  }

  // Row r of J_x(xc, te) and the right-hand side of the mode: -H_t, H or f.
  __device__ __forceinline__ void eval(int emode, double te) {
    G->x[r] = xc;
    wsync();
    cdd xv[N];
#pragma unroll
    for (int j = 0; j < N; ++j) xv[j] = G->x[j];
    wsync();
    // f_r and its gradient: per term the prefix products, then suffix products.
    // A factor of exponent 1 (every factor of a multilinear term) takes x_j
    // itself for its power and its derivative factor 1, instead of products
    // with the double-double one (exact, so the values are the same).
    cdd f = cdd_zero();
    cdd df[N];
#pragma unroll
    for (int j = 0; j < N; ++j) df[j] = cdd_zero();
    for (int tt = t0; tt < t1; ++tt) {
      const uint64_t w = (uint64_t)ex[4 * tt] | ((uint64_t)ex[4 * tt + 1] << 32);
      cdd run = to_cdd({coef[2 * tt], coef[2 * tt + 1]});
      cdd pre[N], pw[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const int e = (int)((w >> (4 * j)) & 15);
        pre[j] = run;
        if (e == 1) {
          pw[j] = xv[j];
          run = cddmul(run, xv[j]);
        } else if (e > 1) {
          cdd p = xv[j];
          for (int k = 1; k < e; ++k) p = cddmul(p, xv[j]);
          pw[j] = p;
          run = cddmul(run, p);
        }
      }
      f = cddadd(f, run);
      cdd suf = {{1.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int mm = 0; mm < N; ++mm) {
        const int m = N - 1 - mm;
        const int e = (int)((w >> (4 * m)) & 15);
        if (e == 1) {
          df[m] = cddadd(df[m], cddmul(pre[m], suf));
          suf = cddmul(suf, pw[m]);
        } else if (e > 1) {
          cdd q = xv[m];
          for (int k = 2; k < e; ++k) q = cddmul(q, xv[m]);
          df[m] = cddadd(df[m], cddmul(cddmul(pre[m], cddscale(q, (double)e)), suf));
          suf = cddmul(suf, pw[m]);
        }
      }
    }
    // start system g_r = x_r^d - 1 and its derivative d x_r^(d-1)
    cdd xr = xv[0];
#pragma unroll
    for (int j = 1; j < N; ++j)
      if (r == j) xr = xv[j];
    cdd pd = {{1.0, 0.0}, {0.0, 0.0}};
    for (int k = 1; k < deg_r; ++k) pd = cddmul(pd, xr);
    const cdd g = cddsub(cddmul(pd, xr), to_cdd({1.0, 0.0}));
    const cdd dg = cddscale(pd, (double)deg_r);
    const cdd gam = to_cdd(gamma);
    const cdd s = cddscale(gam, 1.0 - te);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      A[j] = cddscale(df[j], te);
      if (r == j) A[j] = cddadd(A[j], cddmul(s, dg));
    }
    if (emode == EV_NEG_HT) b = cddsub(cddmul(gam, g), f);
    else if (emode == EV_H) b = cddadd(cddmul(s, g), cddscale(f, te));
    else b = f;
  }

  // Gauss-Jordan on the group's rows: row r of the identity at the end, b
  // the solution component r.  sing: a zero (or NaN) pivot in some column.
  __device__ __forceinline__ cdd solve(bool &sing) {
    sing = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      // pivot row: largest |re| + |im| of the nearest double at or below k
      const cd akk = round_cd(A[k]);
      G->cand[r] = (r >= k) ? fabs(akk.re) + fabs(akk.im) : -1.0;
      wsync();
      int p = k;
      double best = G->cand[k];
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        const double c = G->cand[i];
        if (c > best) {
          best = c;
          p = i;
        }
      }
      if (!(best > 0.0)) sing = true;
      // rows k and p change places through LDS
      if (p != k) {
        if (r == p) {
#pragma unroll
          for (int j = 0; j < N; ++j) G->prow[j] = A[j];
          G->prow[N] = b;
        }
        if (r == k) {
#pragma unroll
          for (int j = 0; j < N; ++j) G->srow[j] = A[j];
          G->srow[N] = b;
        }
      }
      wsync();
      if (p != k) {
        if (r == k) {
#pragma unroll
          for (int j = 0; j < N; ++j) A[j] = G->prow[j];
          b = G->prow[N];
        }
        if (r == p) {
#pragma unroll
          for (int j = 0; j < N; ++j) A[j] = G->srow[j];
          b = G->srow[N];
        }
      }
      wsync();
      // the pivot row, normalised, to every lane of the group
      if (r == k) {
        const cdd inv = cdddiv(to_cdd({1.0, 0.0}), A[k]);
#pragma unroll
        for (int j = 0; j < N; ++j) A[j] = (j == k) ? to_cdd({1.0, 0.0}) : cddmul(A[j], inv);
        b = cddmul(b, inv);
#pragma unroll
        for (int j = 0; j < N; ++j) G->prow[j] = A[j];
        G->prow[N] = b;
      }
      wsync();
      if (r != k) {
        const cdd m = A[k];
#pragma unroll
        for (int j = 0; j < N; ++j)
          A[j] = (j == k) ? cdd_zero() : cddsub(A[j], cddmul(m, G->prow[j]));
        b = cddsub(b, cddmul(m, G->prow[N]));
      }
      wsync();
    }
    return b;
  }

  __device__ __forceinline__ static double cdd_mod(cdd z) {
    const cd v = round_cd(z);
    return sqrt(v.re * v.re + v.im * v.im);
  }
  __device__ __forceinline__ static bool cdd_finite(cdd z) {
    const cd v = round_cd(z);
    return fabs(v.re) < __builtin_inf() && fabs(v.im) < __builtin_inf();
  }

  // One predictor-corrector attempt for TRACK paths, the final Newton for
  // FINAL paths; fin_status >= 0 for paths that end here (endpoint x0).
  __device__ void step(int &fin_status, double &fin_res) {
    const DevTol &tol = a.tol;
    const bool trk = slot && mode == M_TRACK;
    const bool fnl = slot && mode == M_FINAL;
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
    xc = x0;
    int phase = ballot(trk) ? 0 : 4;
    if (phase == 4) iter = fnl;
    for (;;) {
      if (phase == 4 && ballot(iter) == 0) {
        if (trk) {
          ++steps;
          if (ok && conv) {
            t = tn;
            x0 = xc;
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
        if (fnl) x0 = xc;
        nx = group_max(cdd_mod(x0));
        if (trk) {
          if (nx > tol.div_radius) fs = HP_DIVERGED;
          else if (t >= 1.0) mode = M_FINAL;
          else if (h < tol.h_min) fs = HP_FAILED_MINSTEP;
          else if (steps > tol.max_steps) fs = HP_FAILED_MAXSTEPS;
        }
        if (ballot(fs >= 0 || fnl) == 0) break;
        phase = 5;
        xc = x0;
      }
      const double te = (phase == 0) ? (trk ? t : 1.0)
                      : (phase == 1 || phase == 2) ? (trk ? th : 1.0)
                      : (phase == 3 || phase == 4) ? tn : 1.0;
      eval(phase < 4 ? EV_NEG_HT : (phase == 4 ? EV_H : EV_F), te);
      if (phase == 5) {
        res = group_max(cdd_mod(b));
        if (fnl) {
          if (res <= tol.tol_residual && nx <= tol.div_radius) fs = HP_CONVERGED;
          else if (nx > tol.div_radius) fs = HP_DIVERGED;
          else fs = HP_FAILED_NEWTON_T1;
        }
        break;
      }
      bool sing;
      const cdd dx = solve(sing);
      if (phase < 4) {
        // ---- RK4 stage ----
        ok = ok && !sing;
        const double cnext = (phase == 2) ? hs : 0.5 * hs;
        const double wk = (phase == 0 || phase == 3) ? 1.0 : 2.0;
        const cdd k = (phase == 0) ? dx : cddadd(ks, cddscale(dx, wk));
        ks = k;
        xc = (phase == 3) ? cddadd(x0, cddscale(k, hs / 6.0)) : cddadd(x0, cddscale(dx, cnext));
        if (phase == 3) {
          if (trk) {
            evals += 4;
            solves += 4;
          }
          if (fnl) xc = x0;
          iter = (trk && ok) || fnl;
        }
        ++phase;
        continue;
      }
      // ---- Newton iteration: x -= dx ----
      if (iter && !sing) xc = cddsub(xc, dx);
      const double md = group_max(cdd_finite(dx) ? cdd_mod(dx) : __builtin_inf());
      const double mx = group_max(cdd_finite(xc) ? cdd_mod(xc) : __builtin_inf());
      if (iter) {
        ++it;
        ++newton_its;
        ++evals;
        ++solves;
        const bool finite = (md < __builtin_inf()) && (mx < __builtin_inf());
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

  __device__ void write_out(int fs, double res) {
    const long long o = sp->out_path_base + qidx;
    const long long xi = sp->out_x_base + qidx * N + r;
    a.endpoints[xi] = make_double2(x0.re.hi, x0.im.hi);
    a.endpoints_lo[xi] = make_double2(x0.re.lo, x0.im.lo);
    if (r == 0) {
      a.status[o] = fs;
      if (a.stats) {
        hp_path_stats *s = a.stats + o;
        s->steps = steps;
        s->rejections = rejections;
        s->newton_iters = newton_its;
        s->evals = evals;
        s->solves = solves;
        s->pad = 0;
        s->t_final = t;
        s->residual = res;
      }
    }
  }
};

template <int N>
__global__ void __launch_bounds__(64) k_ddtrack(KArgs a) {
  __shared__ DdGroup<N> groups[DdTrack<N>::kGroups + 1];
  DdTrack<N> tr(a, groups);
  const long long npaths = tr.sp->n_paths;
  bool exhausted = false;
  for (;;) {
    // a group whose path is done claims the next one (one atomic per group)
    const bool idle = tr.slot && tr.mode == M_IDLE;
    if (idle && tr.r == 0) tr.G->q = exhausted ? npaths : (long long)atomicAdd(a.qhead, 1ull);
    wsync();
    if (idle) {
      const long long q = tr.G->q;
      if (q < npaths) tr.start_path(q);
      else exhausted = true;
    }
    wsync();
    if (ballot(tr.slot && tr.mode != M_IDLE) == 0) break;
    int fs;
    double res;
    tr.step(fs, res);
    if (tr.slot && fs >= 0) {
      tr.write_out(fs, res);
      tr.mode = M_IDLE;
    }
  }
}

template <int N>
int launch_n(const KArgs &a, int groups, hipStream_t s) {
  hipLaunchKernelGGL(k_ddtrack<N>, dim3((unsigned)groups), dim3(64), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace
}  // namespace hp

int hp_launch_ddtrack(int n, const hp::KArgs &a, int groups, void *stream) {
  using namespace hp;
  hipStream_t s = (hipStream_t)stream;
  switch (n) {
    case 1: return launch_n<1>(a, groups, s);
    case 2: return launch_n<2>(a, groups, s);
    case 3: return launch_n<3>(a, groups, s);
    case 4: return launch_n<4>(a, groups, s);
    case 5: return launch_n<5>(a, groups, s);
    case 6: return launch_n<6>(a, groups, s);
    case 7: return launch_n<7>(a, groups, s);
    case 8: return launch_n<8>(a, groups, s);
    case 9: return launch_n<9>(a, groups, s);
    case 10: return launch_n<10>(a, groups, s);
    case 11: return launch_n<11>(a, groups, s);
    case 12: return launch_n<12>(a, groups, s);
    default: return (int)hipErrorInvalidValue;
  }
}

int hp_ddtrack_per_cu(int n, int *out) {
  *out = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (n) {
#define HP_OCC(K)                                                                         \
  case K:                                                                                 \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, hp::k_ddtrack<K>, 64, 0); \
    break;
    HP_OCC(1) HP_OCC(2) HP_OCC(3) HP_OCC(4) HP_OCC(5) HP_OCC(6)
    HP_OCC(7) HP_OCC(8) HP_OCC(9) HP_OCC(10) HP_OCC(11) HP_OCC(12)
#undef HP_OCC
    default: break;
  }
  return (int)e;
}
