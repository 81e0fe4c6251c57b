// Lane-per-path tracker kernels for gfx950 (CDNA4), complex FP64.
//
// Work mapping.  A workgroup is one 64-lane wavefront and every lane tracks
// its own path (lanes PW..63 stay idle when the LDS of a full wavefront
// would not fit).  The lanes of a wavefront work on one system at a time,
// so the term loop is the same for all of them: term coefficients and
// factor words come in through scalar loads, exponents and variable indices
// are wave-uniform, and only the values differ between lanes.
//
// LDS layout, lane-major: entry e of the wavefront occupies PW * 16 bytes,
// lane l's double2 at byte e * PW * 16 + l * 16.  A wavefront-wide access to
// one entry is one contiguous block, and so is an access where every lane
// picks its own entry (a pivot row), so no access has bank conflicts.
//   entries [0, NMAX * (NMAX + 1)):  [J_x | rhs], row i at i * (NMAX + 1),
//                                    the right-hand side in column NMAX;
//   entries after that:              powers x_v^e, v < n, e = 1 .. emax.
//
// Method (paper: Section 1 and the end of Section 2.1 for independent
// paths and dynamic load balancing).  H(x,t) = gamma (1-t) g(x) + t f(x),
// g_i = x_i^{d_i} - 1.  Each term c x^a is differentiated in reverse mode:
// prefix products from the coefficient, then a backward sweep of suffix
// products that starts from t, so that the partial derivatives arrive
// already scaled by t while the term value stays unscaled (H_t = f - gamma
// g needs f itself).  They are added into the lane's own entries (ds_add_f64:
// no other lane touches them).  The linear systems are solved by LU with
// partial pivoting (largest |re|+|im|, ties to the lowest row) on the LDS
// rows of the lane; row exchanges only swap the row addresses each lane
// keeps in registers.  Step control and the end game are those of the
// library's documented reading (RK4 predictor, Newton corrector, halving /
// doubling step size, final Newton and residual test at t = 1).
//
// Scheduling.  The persistent kernel refills idle lanes from one device
// queue head per system (one atomicAdd per wavefront: ballot, popcount,
// mbcnt), in place of the work crew's guarded next-job pointer (Section 1).
// The plain kernel performs one step per launch for a fixed path -> lane
// map with the path state in HBM.
#include <hip/hip_runtime.h>

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {

// Scalar-loadable (constant address space) views of read-only tables.
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

// N: the number of unknowns, exact (a system of another n runs on another
// instantiation), so every loop over unknowns is unrolled without guards.
template <int N, int PW>
struct Lanes {
  static constexpr int NMAX = N;
  static constexpr int n = N;
  static constexpr int kCols = NMAX + 1;     // J columns + right-hand side
  static constexpr int kEntry = PW * 16;     // bytes of one entry
  static constexpr int kJ = NMAX * kCols;    // entries of [J | rhs]

  const KArgs &a;
  const int lane;
  const bool slot;  // lane holds paths (lane < PW)
  lds_char *base;   // this lane's double2 in entry 0
  // ---- current system (wave-uniform) ----
  cptr<DevSys> sp;
  int emax;
  int deg[NMAX];
  const double2 *tcoef;  // this system's terms (vector loads: their wait
  const uint4 *tmeta;    // counter is not shared with the LDS atomics)
  int kpv[N + 2];  // terms with k factors are this system's terms kpv[k] .. kpv[k+1]-1
  cd gamma;
  long long npaths, out_path_base, out_x_base, id_base;
  const long long *ids;
  // ---- path state ----
  int mode, accepts, steps, rejections, newton_its, evals, solves;
  long long qidx;
  double t, h;
  cd x0[NMAX], xc[NMAX], ks[NMAX];

  __device__ Lanes(const KArgs &args, char *smem)
      : a(args), lane(threadIdx.x & 63), slot((threadIdx.x & 63) < PW) {
    base = (lds_char *)smem + (slot ? lane : 0) * 16;
    mode = M_IDLE;
    t = h = 0.0;
    qidx = 0;
    accepts = steps = rejections = newton_its = evals = solves = 0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) x0[i] = xc[i] = ks[i] = {0.0, 0.0};
  }

  // ---- LDS entries of this lane ----
  __device__ __forceinline__ lds_char *ent(int e) const { return base + e * kEntry; }
  __device__ __forceinline__ lds_char *jent(int i, int j) const { return ent(i * kCols + j); }
  __device__ __forceinline__ lds_char *xpent(int v, int e1) const { return ent(kJ + v * emax + e1); }

  __device__ __forceinline__ void load_system(int s) {
    sp = as_const(a.sys) + s;
    emax = sp->emax;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) deg[i] = (i < n) ? sp->deg[i] : 1;
    tcoef = a.tcoef + sp->term_base;
    tmeta = a.tmeta + sp->term_base;
    {
      cptr<int32_t> kp = as_const(a.eqp) + sp->eq_base;
#pragma unroll
      for (int k = 0; k <= N + 1; ++k) kpv[k] = kp[k < N + 1 ? k : HP_MAX_N + 1];
    }
    gamma = {sp->gre, sp->gim};
    npaths = sp->n_paths;
    out_path_base = sp->out_path_base;
    out_x_base = sp->out_x_base;
    ids = (const long long *)sp->ids;
    id_base = sp->id_base;
  }

  // ------------------------------------------------------------------ eval
  // One term as loaded: coefficient and factor word.
  struct Term {
    cd c;
    uint32_t w[4];
  };
  __device__ __forceinline__ Term load_term(int tt) const {
    const double2 cc = tcoef[tt];
    const uint4 mw = tmeta[tt];
    return {{cc.x, cc.y}, {mw.x, mw.y, mw.z, mw.w}};
  }
  // Factor m of a term: variable (low nibble) and exponent (high nibble).
  __device__ __forceinline__ static int factor_byte(const Term &T, int m) {
    return (T.w[(m + 1) >> 2] >> (8 * ((m + 1) & 3))) & 0xff;
  }

  // Terms with exactly K factors, all lanes on the same term, software
  // pipelined: the factor words of term tt + 2 are in flight and the
  // powers of term tt + 1 are read while term tt is differentiated, and
  // those reads are issued before the atomics of term tt, so that waiting
  // for them never waits for the atomics.
  template <int K>
  __device__ __forceinline__ void terms_k(int lo, int hi, double te) {
    if constexpr (K == 0) {
      // constant terms: f_eq += c
#pragma nounroll
      for (int tt = lo; tt < hi; ++tt) {
        const Term T = load_term(tt);
        addl(jent((int)(T.w[3] >> 24), NMAX), T.c);
      }
    } else {
      terms_pipelined<K>(lo, hi, te);
    }
  }
  template <int K>
  __device__ __forceinline__ void terms_pipelined(int lo, int hi, double te) {
    const int last = hi - 1;
    Term cur = load_term(lo);
    Term nxt = load_term(lo + 1 < hi ? lo + 1 : last);
    cd phi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const int b = factor_byte(cur, m);
      phi[m] = ldl(xpent(b & 15, (b >> 4) - 1));
    }
#pragma nounroll
    for (int tt = lo; tt < hi; ++tt) {
      const Term nn = load_term(tt + 2 <= last ? tt + 2 : last);
      // powers of the next term (the current one again past the end)
      cd phn[K];
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const int b = factor_byte(nxt, m);
        phn[m] = ldl(xpent(b & 15, (b >> 4) - 1));
      }
      const int eq = (int)(cur.w[3] >> 24);
      lds_char *frow = jent(eq, 0);
      {
        cd P[K];
        cd run = cur.c;
#pragma unroll
        for (int m = 0; m < K; ++m) {
          run = cmul(run, phi[m]);
          P[m] = run;
        }
        addl(frow + NMAX * kEntry, run);  // f_eq, unscaled
        // backward sweep; S starts at t, so every partial comes out times t
        cd S = {te, 0.0};
#pragma unroll
        for (int m = K - 1; m >= 0; --m) {
          const int b = factor_byte(cur, m);
          const int v = b & 15, e = b >> 4;
          const cd left = (m == 0) ? cur.c : P[m > 0 ? m - 1 : 0];
          cd d = (m == K - 1) ? cscale(left, te) : cmul(left, S);
          if (e > 1) {
            // the power e-1 of x_v, times e
            const cd q = ldl(xpent(v, e - 2));
            d = cmul(d, cscale(q, (double)e));
          }
          addl(frow + v * kEntry, d);
          if (m > 0) S = (m == K - 1) ? cscale(phi[m], te) : cmul(S, phi[m]);
        }
      }
      cur = nxt;
      nxt = nn;
#pragma unroll
      for (int m = 0; m < K; ++m) phi[m] = phn[m];
    }
  }

  template <int K>
  __device__ __forceinline__ void terms_upto(double te) {
    if constexpr (K >= 0) {
      terms_upto<K - 1>(te);
      const int lo = kpv[K], hi = kpv[K + 1];
      if (lo < hi) terms_k<K>(lo, hi, te);
    }
  }

  // [J_x(xc, te) | rhs] into the lane's entries; rhs is -H_t (EV_NEG_HT),
  // H (EV_H) or f (EV_F) at (xc, te).
  __device__ __forceinline__ void eval(int emode, double te) {
#pragma unroll
    for (int v = 0; v < NMAX; ++v) {
      if (v < n) {
        cd p = xc[v];
        stl(xpent(v, 0), p);
        for (int e = 2; e <= emax; ++e) {
          p = cmul(p, xc[v]);
          stl(xpent(v, e - 1), p);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
          if (j < n) stl(jent(i, j), {0.0, 0.0});
        stl(jent(i, NMAX), {0.0, 0.0});
      }
    }
    terms_upto<NMAX>(te);
    // start system part: J_ii += s d_i x_i^{d_i-1}; right-hand side
    const cd s = cscale(gamma, 1.0 - te);
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n) {
        const int d = deg[i];
        cd xq = {1.0, 0.0};
        for (int e = 1; e < d; ++e) xq = cmul(xq, xc[i]);
        cd g = cmul(xq, xc[i]);
        g.re -= 1.0;
        const cd sdg = cmul(s, cscale(xq, (double)d));
        stl(jent(i, i), cadd(ldl(jent(i, i)), sdg));
        const cd f = ldl(jent(i, NMAX));
        const cd hv = cadd(cmul(s, g), cscale(f, te));
        const cd mht = csub(cmul(gamma, g), f);
        stl(jent(i, NMAX), csel(emode == EV_F, f, csel(emode == EV_H, hv, mht)));
      }
    }
  }

  // ----------------------------------------------------------------- solve
  // LU with partial pivoting of the lane's [J | rhs], then back
  // substitution into dx.  sing: an exactly zero (or NaN) pivot.  The next
  // pivot column is updated first and kept in registers (look-ahead), so the
  // pivot search never waits on LDS; the other columns are streamed: column
  // j + 1 is read before column j is written back.
  __device__ __forceinline__ void solve(cd dx[NMAX], bool &sing) {
    lds_char *row[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) row[i] = base + i * kCols * kEntry;
    sing = false;
    cd col[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) col[i] = ldl(row[i]);
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k < n) {
        double best = -1.0;
        int p = k;
#pragma unroll
        for (int i = k; i < NMAX; ++i) {
          if (i < n) {
            const double c = cabs1(col[i]);
            const bool take = c > best;
            best = take ? c : best;
            p = take ? i : p;
          }
        }
        if (!(best > 0.0)) sing = true;
        // exchange logical rows k and p (row addresses and column values)
        lds_char *rk = row[k];
        cd ck = col[k];
#pragma unroll
        for (int i = k + 1; i < NMAX; ++i) {
          if (i < n) {
            const bool sw = (i == p);
            lds_char *ri = row[i];
            const cd ci = col[i];
            row[i] = sw ? row[k] : ri;
            col[i] = csel(sw, col[k], ci);
            rk = sw ? ri : rk;
            ck = csel(sw, ci, ck);
          }
        }
        row[k] = rk;
        const cd inv = crecip_nr(ck);
        stl(row[k] + k * kEntry, inv);  // kept for the back substitution
#pragma unroll
        for (int i = k + 1; i < NMAX; ++i)
          if (i < n) col[i] = cmul(col[i], inv);  // multipliers
        // look-ahead: column k + 1 of the remaining rows, into registers
        cd nxt[NMAX];
        if (k + 1 < n) {
          const cd u = ldl(row[k] + (k + 1) * kEntry);
          cd av[NMAX];
#pragma unroll
          for (int i = k + 1; i < NMAX; ++i)
            if (i < n) av[i] = ldl(row[i] + (k + 1) * kEntry);
#pragma unroll
          for (int i = k + 1; i < NMAX; ++i)
            if (i < n) nxt[i] = cfms(av[i], col[i], u);
        }
        // the other columns k+2 .. n-1 and the right-hand side, streamed
        cd pa[NMAX], pu = {0.0, 0.0};
        int pj = -1;
#pragma unroll
        for (int j = k + 2; j <= NMAX; ++j) {
          if (j < n || j == NMAX) {
            const cd u = ldl(row[k] + j * kEntry);
            cd av[NMAX];
#pragma unroll
            for (int i = k + 1; i < NMAX; ++i)
              if (i < n) av[i] = ldl(row[i] + j * kEntry);
            if (pj >= 0) {
#pragma unroll
              for (int i = k + 1; i < NMAX; ++i)
                if (i < n) stl(row[i] + pj * kEntry, cfms(pa[i], col[i], pu));
            }
#pragma unroll
            for (int i = k + 1; i < NMAX; ++i)
              if (i < n) pa[i] = av[i];
            pu = u;
            pj = j;
          }
        }
        if (pj >= 0) {
#pragma unroll
          for (int i = k + 1; i < NMAX; ++i)
            if (i < n) stl(row[i] + pj * kEntry, cfms(pa[i], col[i], pu));
        }
#pragma unroll
        for (int i = k + 1; i < NMAX; ++i)
          if (i < n) col[i] = nxt[i];
      }
    }
#pragma unroll
    for (int k = NMAX - 1; k >= 0; --k) {
      if (k < n) {
        cd y = ldl(row[k] + NMAX * kEntry);
#pragma unroll
        for (int j = k + 1; j < NMAX; ++j)
          if (j < n) y = cfms(y, ldl(row[k] + j * kEntry), dx[j]);
        dx[k] = cmul(y, ldl(row[k] + k * kEntry));
      } else {
        dx[k] = {0.0, 0.0};
      }
    }
  }

  // ------------------------------------------------------------ start path
  __device__ __forceinline__ void start_path(long long q) {
    qidx = q;
    const long long pid = ids ? ids[q] : id_base + q;
    cptr<double> roots = as_const((const double *)a.roots) + 2 * sp->root_base;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n) {
        const long long kk = (pid / sp->radix[i]) % deg[i];
        const int ri = sp->root_off[i] + (int)kk;
        x0[i] = {roots[2 * ri], roots[2 * ri + 1]};
      }
    }
    mode = M_TRACK;
    t = 0.0;
    h = a.tol.h_init;
    accepts = steps = rejections = newton_its = evals = solves = 0;
  }

  __device__ __forceinline__ double vmax_mod(const cd v[NMAX]) const {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) m = nmax(m, cmod(v[i]));
    return m;
  }

  // ------------------------------------------------------------- one step
  // One predictor-corrector attempt for TRACK paths, the final Newton for
  // FINAL paths; fin_status >= 0 for paths that end here (endpoint x0).
  // Phases, each one evaluation and (except 5) one solve:
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
    for (int i = 0; i < NMAX; ++i) xc[i] = x0[i];
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
            for (int i = 0; i < NMAX; ++i) x0[i] = xc[i];
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
          for (int i = 0; i < NMAX; ++i) x0[i] = xc[i];
        }
        nx = vmax_mod(x0);
        if (trk) {
          if (nx > tol.div_radius) fs = HP_DIVERGED;
          else if (t >= 1.0) mode = M_FINAL;
          else if (h < tol.h_min) fs = HP_FAILED_MINSTEP;
          else if (steps > tol.max_steps) fs = HP_FAILED_MAXSTEPS;
        }
        if (ballot(fs >= 0 || fnl) == 0) break;
        phase = 5;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) xc[i] = x0[i];
      }
      const double te = (phase == 0) ? (trk ? t : 1.0)
                      : (phase == 1 || phase == 2) ? (trk ? th : 1.0)
                      : (phase == 3 || phase == 4) ? tn : 1.0;
      eval(phase < 4 ? EV_NEG_HT : (phase == 4 ? EV_H : EV_F), te);
      if (phase == 5) {
        // ---- residual ||f(x0)||_inf of ending paths, classification ----
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
          if (i < n) r = nmax(r, cmod(ldl(jent(i, NMAX))));
        res = r;
        if (fnl) {
          if (res <= tol.tol_residual && nx <= tol.div_radius) fs = HP_CONVERGED;
          else if (nx > tol.div_radius) fs = HP_DIVERGED;
          else fs = HP_FAILED_NEWTON_T1;
        }
        break;
      }
      bool sing;
      cd dsl[NMAX];
      solve(dsl, sing);
      if (phase < 4) {
        // ---- RK4 stage ----
        ok = ok && !sing;
        const double cnext = (phase == 2) ? hs : 0.5 * hs;
        const double wk = (phase == 0 || phase == 3) ? 1.0 : 2.0;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          ks[i] = csel(phase == 0, dsl[i], cadd(ks[i], cscale(dsl[i], wk)));
          xc[i] = csel(phase == 3, cadd(x0[i], cscale(ks[i], hs / 6.0)),
                       cadd(x0[i], cscale(dsl[i], cnext)));
        }
        if (phase == 3) {
          if (trk) {
            evals += 4;
            solves += 4;
          }
          if (fnl) {
#pragma unroll
            for (int i = 0; i < NMAX; ++i) xc[i] = x0[i];
          }
          iter = (trk && ok) || fnl;
        }
        ++phase;
        continue;
      }
      // ---- Newton iteration: x -= dx ----
      if (iter && !sing) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i) xc[i] = csub(xc[i], dsl[i]);
      }
      const double md = vmax_mod(dsl), mx = vmax_mod(xc);
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

  __device__ __forceinline__ void write_out(int fs, double res) {
    double2 *e = a.endpoints + out_x_base + qidx * n;
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) e[i] = make_double2(x0[i].re, x0[i].im);
    const long long o = out_path_base + qidx;
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
};

// ------------------------------------------------------------------------
// Persistent kernel: resident wavefronts loop until every system's queue is
// drained; a wavefront moves to the next system once its queue is empty and
// its own lanes are idle.
// ------------------------------------------------------------------------
template <int N, int PW>
__global__ void __launch_bounds__(64) k_lanes(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Lanes<N, PW> tr(a, smem);
  const int first_sys = blockIdx.x % a.n_systems;
  for (int v = 0; v < a.n_systems; ++v) {
    const int s = (first_sys + v) % a.n_systems;
    tr.load_system(s);
    bool exhausted = false;
    for (;;) {
      // ---- refill idle lanes: one atomic per wavefront ----
      const bool idle = tr.slot && tr.mode == M_IDLE;
      const uint64_t m = ballot(idle);
      if (m != 0 && !exhausted) {
        const unsigned cnt = __popcll(m);
        const int first = __builtin_ctzll(m);
        unsigned long long qb = 0;
        if (tr.lane == first) qb = atomicAdd(&a.qhead[s], (unsigned long long)cnt);
        qb = __shfl(qb, first);
        const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (idle) {
          const long long q = (long long)qb + rank;
          if (q < tr.npaths) tr.start_path(q);
        }
        if ((long long)(qb + cnt) >= tr.npaths) exhausted = true;
      }
      if (ballot(tr.mode != M_IDLE) == 0) {
        if (exhausted) break;  // this system is drained for this wavefront
        continue;
      }
      // lanes past PW hold no LDS column: they sit out the step
      if (tr.slot) {
        int fs;
        double res;
        tr.step(fs, res);
        if (fs >= 0) {
          tr.write_out(fs, res);
          tr.mode = M_IDLE;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------
// Plain tracker: one step per launch.  Wavefront b owns queue indices
// [PW b, PW b + PW) of system 0; path state lives in HBM between launches
// (initialised by k_plain_init).
// ------------------------------------------------------------------------
template <int N, int PW>
__global__ void __launch_bounds__(64) k_lanes_plain(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Lanes<N, PW> tr(a, smem);
  tr.load_system(0);
  const long long P = a.ps.P;
  const long long q = (long long)blockIdx.x * PW + tr.lane;
  const bool valid = tr.slot && q < tr.npaths;
  const int md = valid ? a.ps.iv[q] : (int)M_IDLE;
  if (ballot(md != M_IDLE) == 0) return;
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
    for (int i = 0; i < N; ++i) {
      const double2 z = a.ps.x0[i * P + q];
      tr.x0[i] = {z.x, z.y};
    }
  }
  if (tr.slot) {
    int fs;
    double res;
    tr.step(fs, res);
    if (fs >= 0) {
      tr.write_out(fs, res);
      tr.mode = M_IDLE;
    }
  }
  if (md != M_IDLE) {
#pragma unroll
    for (int i = 0; i < N; ++i) a.ps.x0[i * P + q] = make_double2(tr.x0[i].re, tr.x0[i].im);
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
  const uint64_t m = ballot(tr.mode != M_IDLE && valid);
  if (tr.lane == 0 && m) atomicAdd(a.ps.active, (unsigned)__popcll(m));
}

}  // namespace hp

// ------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------
using namespace hp;

template <class K>
static int lanes_allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return (int)hipSuccess;
  return (int)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
}

template <int NMAX, int PW>
static int lanes_persistent_t(const KArgs &a, int groups, size_t lds, hipStream_t s) {
  int rc = lanes_allow_lds(k_lanes<NMAX, PW>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_lanes<NMAX, PW>), dim3(groups), dim3(64), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, int PW>
static int lanes_plain_t(const KArgs &a, int groups, size_t lds, hipStream_t s) {
  int rc = lanes_allow_lds(k_lanes_plain<NMAX, PW>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_lanes_plain<NMAX, PW>), dim3(groups), dim3(64), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, int PW>
static int lanes_occupancy_t(size_t lds, int *out) {
  int rc = lanes_allow_lds(k_lanes<NMAX, PW>, lds);
  if (rc) return rc;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_lanes<NMAX, PW>, 64, lds);
}

#define HP_LANES_DISPATCH(NN, PWV, CALL)          \
  switch ((NN) * 1000 + (PWV)) {                  \
    case 1064: return CALL(1, 64);                \
    case 2064: return CALL(2, 64);                \
    case 3064: return CALL(3, 64);                \
    case 4064: return CALL(4, 64);                \
    case 5064: return CALL(5, 64);                \
    case 6064: return CALL(6, 64);                \
    case 7064: return CALL(7, 64);                \
    case 8064: return CALL(8, 64);                \
    case 7032: return CALL(7, 32);                \
    case 8032: return CALL(8, 32);                \
    default: return (int)hipErrorInvalidValue;    \
  }

int hp_launch_lanes(int n, int pw, const KArgs &a, int groups, size_t lds, void *stream) {
#define CALLP(N, W) lanes_persistent_t<N, W>(a, groups, lds, (hipStream_t)stream)
  HP_LANES_DISPATCH(n, pw, CALLP)
#undef CALLP
}

int hp_launch_lanes_plain(int n, int pw, const KArgs &a, int groups, size_t lds, void *stream) {
#define CALLS(N, W) lanes_plain_t<N, W>(a, groups, lds, (hipStream_t)stream)
  HP_LANES_DISPATCH(n, pw, CALLS)
#undef CALLS
}

int hp_lanes_per_cu(int n, int pw, size_t lds, int *out) {
#define CALLO(N, W) lanes_occupancy_t<N, W>(lds, out)
  HP_LANES_DISPATCH(n, pw, CALLO)
#undef CALLO
}
