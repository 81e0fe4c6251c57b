// Batched homotopy path tracker kernels for gfx950 (CDNA4), complex FP64.
//
// Work mapping.  A workgroup is one 64-lane wavefront.  A path is handled by
// a group of n consecutive lanes (n = number of unknowns): lane r of the
// group owns equation r (row r of the Jacobian) and unknown r of the path
// state; a wavefront carries floor(64 / n) paths.  Everything a path needs
// is exchanged through the group's LDS region and never crosses wavefronts,
// so no cross-wave barrier is involved; the __syncthreads() calls below only
// order the LDS accesses of the single wavefront.
//
// Method.  H(x,t) = gamma(1-t) g(x) + t f(x), g_i = x_i^{d_i} - 1 (paper:
// Section 1 and the end of Section 2.1 for independent paths and dynamic load
// balancing).  f and its Jacobian are evaluated by reverse-mode algorithmic
// differentiation of each monomial: prefix products with the coefficient
// folded in, then a backward sweep of suffix products.  The host sorts all
// terms of a system by their number of factors k; the lanes of a group take
// consecutive terms of one k at a time, so every lane runs the same
// straight-line code, and add the partial derivatives into the path's
// Jacobian in LDS (ds_add_f64), whose real and imaginary parts are separate
// planes so that the 8-byte atomics of a group's lanes spread over the
// banks.  Linear systems are solved by Gauss-Jordan
// elimination with partial pivoting (largest |re|+|im| in the column, ties
// to the lowest row), one row per lane: the pivot search is a DPP butterfly
// in registers when the groups are aligned (n = 2, 4, 8), else an exchange
// through LDS; the normalised pivot row goes through LDS.  One RK4 predictor step and up to max_newton Newton
// iterations form a step; the step control and the final Newton at t = 1
// follow the library's documented reading.
//
// Scheduling.  The persistent kernel replaces the work crew's guarded
// next-job pointer (Section 1) with a device atomic queue head per system:
// after every step, groups whose path finished claim new path ids with one
// atomicAdd per wavefront (ballot / popcount / mbcnt).  The plain kernel
// performs one step per launch for a fixed path -> group map.
#include <hip/hip_runtime.h>

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {

// One butterfly step of a (value, index) max over aligned lane groups,
// ties to the lowest index: read the DPP partner's pair, keep the larger.
// CTRL: quad_perm [1,0,3,2] (0xB1, lane ^ 1), quad_perm [2,3,0,1] (0x4E,
// lane ^ 2) or row_half_mirror (0x141, lane 7 - lane within 8).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)bits, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(bits >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ double dpp_max_step(double v, int &idx) {
  const double ov = dpp_double<CTRL>(v);
  const int oi = __builtin_amdgcn_mov_dpp(idx, CTRL, 0xf, 0xf, false);
  const bool take = (ov > v) || (ov == v && oi < idx);
  idx = take ? oi : idx;
  return take ? ov : v;
}

// GEN: the general start system / explicit start point code is compiled in
// (a separate instantiation, so that the total-degree kernels do not carry
// its registers).
template <int NMAX, bool GEN>
struct Tracker {
  const KArgs &a;
  const int lane;
  char *smem;
  // ---- current system (wave-uniform) ----
  int n, emax, ngroups;
  const DevSys *sp;
  const double2 *gcoef;  // this system's terms in global memory
  const uint4 *gmeta;
  bool staged;           // terms copied to LDS (right after the refill area)
  int nterms;
  // terms with k factors are this system's terms kp[k] .. kp[k+1]-1; cached
  // in registers for the narrow variants (the wide ones would spill)
  static constexpr bool kCacheKp = NMAX <= 8;
  int kpv[NMAX + 2];
  const int *kpm;
  // general start system g (terms in global memory) and explicit start points
  bool has_g;
  const int *gkpm;
  const double2 *ggcoef;
  const uint4 *ggmeta;
  const double2 *start;
  cd gamma;
  long long npaths, out_path_base, out_x_base, id_base;
  const long long *ids;
  // ---- lane role ----
  int grp, r;   // group (path slot) and row / unknown index within it
  int deg_r;    // degree of equation r
  bool leader;  // r == 0 of a real group
  // ---- LDS region of this lane's group (compile-time strides) ----
  GroupLds<NMAX> *G;
  double *Jrr, *Jri;  // own row of the Jacobian accumulator (real, imaginary)
  double2 *xp;    // [n][emax] powers x_v^e, e = 1..emax (after the fixed part)
  long long *ctl; // [64] refill broadcast (wave-wide)
  // ---- per-path state (replicated in the group's lanes) ----
  int mode, accepts, steps, rejections, newton_its, evals, solves;
  long long qidx;
  double t, h;
  // ---- own unknown r ----
  cd x0, xc, ks;
  // ---- own row r of [J | b] ----
  cd A[NMAX];
  cd b;

  __device__ Tracker(const KArgs &args, char *s) : a(args), lane(threadIdx.x & 63), smem(s) {
    ctl = (long long *)smem;
    mode = M_IDLE;
    t = h = 0.0;
    qidx = 0;
    accepts = steps = rejections = newton_its = evals = solves = 0;
    x0 = xc = ks = b = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NMAX; ++j) A[j] = {0.0, 0.0};
  }

  __device__ __forceinline__ void load_system(int s) {
    sp = a.sys + s;
    n = sp->n;
    emax = sp->emax;
    ngroups = kLanes / n;
    kpm = a.eqp + sp->eq_base;
    if constexpr (kCacheKp) {
#pragma unroll
      for (int k = 0; k <= NMAX + 1; ++k) kpv[k] = kpm[k < NMAX + 1 ? k : HP_MAX_N + 1];
    }
    has_g = sp->g_n_terms > 0;
    ggcoef = a.tcoef + sp->g_term_base;
    ggmeta = a.tmeta + sp->g_term_base;
    gkpm = a.eqp + sp->g_eq_base;
    start = sp->start;
    // stage a small term table in LDS (all lanes copy, then order)
    const int nt = sp->n_terms;
    size_t tbytes = 0;
    gcoef = a.tcoef + sp->term_base;
    gmeta = a.tmeta + sp->term_base;
    nterms = nt;
    staged = a.stage && nt <= kMaxStagedTerms;
    if (staged) {
      double2 *sc = staged_coef();
      uint4 *sm = staged_meta();
      wsync();
      for (int i = lane; i < nt; i += kLanes) {
        sc[i] = gcoef[i];
        sm[i] = gmeta[i];
      }
      wsync();
      tbytes = (size_t)nt * 32;
    }
    gamma = {sp->gre, sp->gim};
    npaths = sp->n_paths;
    out_path_base = sp->out_path_base;
    out_x_base = sp->out_x_base;
    ids = (const long long *)sp->ids;
    id_base = sp->id_base;
    grp = lane / n;  // lanes past the last full group form a spare group
    r = lane - grp * n;
    leader = (r == 0) && grp < ngroups;
    deg_r = sp->deg[r < n ? r : 0];
    char *g = smem + kCtlBytes + tbytes + (size_t)grp * group_lds_bytes(NMAX, emax);
    G = (GroupLds<NMAX> *)g;
    Jrr = &G->Jre[r][0];
    Jri = &G->Jim[r][0];
    xp = (double2 *)(g + sizeof(GroupLds<NMAX>));
  }

  // staged term table (LDS address space: plain ds_read)
  __device__ __forceinline__ double2 *staged_coef() const { return (double2 *)(smem + kCtlBytes); }
  __device__ __forceinline__ uint4 *staged_meta() const {
    return (uint4 *)(smem + kCtlBytes + (size_t)nterms * sizeof(double2));
  }

  // max over the lanes of this lane's group (reads are unconditional so
  // that they issue back to back; entries past n are masked afterwards)
  __device__ __forceinline__ double group_max(double v) {
    G->red[r] = v;
    wsync();
    double x[NMAX];
#pragma unroll
    for (int q = 0; q < NMAX; ++q) x[q] = G->red[q];
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < NMAX; ++q) m = (q < n) ? nmax(m, x[q]) : m;
    wsync();
    return m;
  }
  __device__ __forceinline__ void group_max2(double &u, double &v) {
    G->red[r] = u;
    G->red[NMAX + r] = v;
    wsync();
    double x[NMAX], y[NMAX];
#pragma unroll
    for (int q = 0; q < NMAX; ++q) {
      x[q] = G->red[q];
      y[q] = G->red[NMAX + q];
    }
    double mu = 0.0, mv = 0.0;
#pragma unroll
    for (int q = 0; q < NMAX; ++q) {
      mu = (q < n) ? nmax(mu, x[q]) : mu;
      mv = (q < n) ? nmax(mv, y[q]) : mv;
    }
    wsync();
    u = mu;
    v = mv;
  }

  // ------------------------------------------------------------------ eval
  // Groups of 2, 4 or 8 aligned lanes: cross-lane sums and maxima in
  // registers (DPP) instead of LDS.
  __device__ __forceinline__ bool dpp_groups() const {
    return n == 2 || n == 4 || (n == 8 && NMAX >= 8);
  }

  // Sum of v over this lane's group (DPP butterfly: xor 1, xor 2 within
  // quads, mirror within 8 lanes); every lane of the wave must be active.
  __device__ __forceinline__ cd group_sum_dpp(cd v) {
    v.re += dpp_double<0xB1>(v.re);
    v.im += dpp_double<0xB1>(v.im);
    if (n >= 4) {
      v.re += dpp_double<0x4E>(v.re);
      v.im += dpp_double<0x4E>(v.im);
    }
    if (n >= 8) {
      v.re += dpp_double<0x141>(v.re);
      v.im += dpp_double<0x141>(v.im);
    }
    return v;
  }

  // Adds the term values of one chunk (the n consecutive terms a group takes
  // at once) into vt[eq] for DPP-aligned groups.  When every chunk of the
  // wave lies in one equation (the host flags such chunks), the group sums
  // its values in registers and lane 0 makes the one LDS add; otherwise
  // every lane with a term adds its own (same-address atomics serialise).
  __device__ __forceinline__ void add_values(bool act, bool uni, int eq, cd v, double *vre,
                                             double *vim) {
    if (ballot(act && !uni) == 0) {
      v = group_sum_dpp(v);
      if (act && r == 0) lds_add2(&vre[eq], &vim[eq], v);
    } else if (act) {
      lds_add2(&vre[eq], &vim[eq], v);
    }
  }

  // One term c * prod phi_m: partials times sigma go to J[eq][.]; the value
  // goes to vt[eq] (DV false) or is returned for add_values (DV true).
  template <int K, bool CPLX, bool DV>
  __device__ __forceinline__ cd one_term(const double2 cc, const uint4 mw, cd sigma,
                                         double *vre, double *vim) {
    const uint32_t w[4] = {mw.x, mw.y, mw.z, mw.w};
    const cd c = {cc.x, cc.y};
    const int eq = (int)(w[3] >> 24);
    if constexpr (K == 0) {
      if constexpr (!DV) lds_add2(&vre[eq], &vim[eq], c);
      return c;
    } else {
      int vv[K], ee[K];
      cd P[K], phi[K];
      cd run = c;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const int byte = (w[(m + 1) >> 2] >> (8 * ((m + 1) & 3))) & 0xff;
        ee[m] = byte >> 4;
        vv[m] = byte & 15;
        phi[m] = ld(&xp[vv[m] * emax + ee[m] - 1]);
      }
#pragma unroll
      for (int m = 0; m < K; ++m) {
        run = cmul(run, phi[m]);
        P[m] = run;
      }
      if constexpr (!DV) lds_add2(&vre[eq], &vim[eq], run);
      double *jre = &G->Jre[eq][0];
      double *jim = &G->Jim[eq][0];
      cd S = sigma;
#pragma unroll
      for (int m = K - 1; m >= 0; --m) {
        const cd left = (m == 0) ? c : P[m > 0 ? m - 1 : 0];
        cd d = CPLX ? cmul(left, S) : (m == K - 1 ? cscale(left, S.re) : cmul(left, S));
        if (ee[m] > 1) {
          const cd q = ld(&xp[vv[m] * emax + ee[m] - 2]);
          d = cmul(d, cscale(q, (double)ee[m]));
        }
        lds_add2(&jre[vv[m]], &jim[vv[m]], d);
        if (m > 0) S = (m == K - 1 && !CPLX) ? cscale(phi[m], S.re) : cmul(S, phi[m]);
      }
      return run;
    }
  }

  // Terms with exactly K factors: this lane takes terms lo + r, lo + r + n, ...
  // Term values go to vt[eq] unscaled; partial derivatives go to J[eq][v]
  // times sigma (the backward sweep starts from sigma): sigma = t for f
  // (CPLX false: real) and gamma (1 - t) for a general start system g.
  // From the staged table (LDS) a term is read where it is used; from global
  // memory (large systems: many terms of at most a few factors per class)
  // the lane's next term is read while this one is processed.
  template <int K, bool LDS, bool CPLX, bool DV>
  __device__ __forceinline__ void terms_k(int lo, int hi, const double2 *gc, const uint4 *gm,
                                          cd sigma, double *vre, double *vim) {
    if constexpr (LDS || K > 4) {
      const double2 *tcoef = LDS ? staged_coef() : gc;
      const uint4 *tmeta = LDS ? staged_meta() : gm;
#pragma nounroll
      for (int base = lo; base < hi; base += n) {
        const int tt = base + r;
        const bool act = tt < hi;
        if constexpr (DV) {
          cd v = {0.0, 0.0};
          uint4 mw = {0u, 0u, 0u, 0u};
          if (act) {
            mw = tmeta[tt];
            v = one_term<K, CPLX, true>(tcoef[tt], mw, sigma, vre, vim);
          }
          add_values(act, (mw.x & kChunkUniform) != 0, (int)(mw.w >> 24), v, vre, vim);
        } else {
          if (act) one_term<K, CPLX, false>(tcoef[tt], tmeta[tt], sigma, vre, vim);
        }
      }
    } else {
      const int last = hi - 1;
      int ti = lo + r < last ? lo + r : last;
      double2 pc = gc[ti];
      uint4 pm = gm[ti];
#pragma nounroll
      for (int base = lo; base < hi; base += n) {
        const int tt = base + r;
        const double2 cc = pc;
        const uint4 mw = pm;
        ti = tt + n < last ? tt + n : last;
        pc = gc[ti];
        pm = gm[ti];
        const bool act = tt < hi;
        if constexpr (DV) {
          cd v = {0.0, 0.0};
          if (act) v = one_term<K, CPLX, true>(cc, mw, sigma, vre, vim);
          add_values(act, (mw.x & kChunkUniform) != 0, (int)(mw.w >> 24), v, vre, vim);
        } else {
          if (act) one_term<K, CPLX, false>(cc, mw, sigma, vre, vim);
        }
      }
    }
  }

  template <int K, bool LDS, bool CPLX, bool DV>
  __device__ __forceinline__ void terms_upto(const int *kk, const double2 *gc, const uint4 *gm,
                                             cd sigma, double *vre, double *vim) {
    if constexpr (K >= 0) {
      terms_upto<K - 1, LDS, CPLX, DV>(kk, gc, gm, sigma, vre, vim);
      const int lo = kk[K], hi = kk[K + 1];
      if (lo < hi) terms_k<K, LDS, CPLX, DV>(lo, hi, gc, gm, sigma, vre, vim);
    }
  }

  // Own row of J_x(xc, te) into A and, in b: -H_t (EV_NEG_HT), H (EV_H) or
  // f (EV_F) at (xc, te).
  __device__ __forceinline__ void eval(int emode, double te) {
    const cd s = cscale(gamma, 1.0 - te);
    // powers of the own unknown; zero the own row of the accumulators
    {
      cd p = xc;
      st(&xp[r * emax], p);
      for (int e = 2; e <= emax; ++e) {
        p = cmul(p, xc);
        st(&xp[r * emax + e - 1], p);
      }
#pragma unroll
      for (int j = 0; j < NMAX; ++j) {
        Jrr[j] = 0.0;
        Jri[j] = 0.0;
      }
      G->fre[r] = 0.0;
      G->fim[r] = 0.0;
      if constexpr (GEN) {
        G->gre[r] = 0.0;
        G->gim[r] = 0.0;
      }
    }
    wsync();
    const cd tsig = {te, 0.0};
    const int *kk = kCacheKp ? kpv : kpm;
    // DPP value sums only where the groups are aligned (wave-uniform choice)
    if (dpp_groups()) {
      if (staged) terms_upto<NMAX, true, false, true>(kk, gcoef, gmeta, tsig, G->fre, G->fim);
      else terms_upto<NMAX, false, false, true>(kk, gcoef, gmeta, tsig, G->fre, G->fim);
    } else {
      if (staged) terms_upto<NMAX, true, false, false>(kk, gcoef, gmeta, tsig, G->fre, G->fim);
      else terms_upto<NMAX, false, false, false>(kk, gcoef, gmeta, tsig, G->fre, G->fim);
    }
    if constexpr (GEN) {
      if (has_g) terms_upto<NMAX, false, true, false>(gkpm, ggcoef, ggmeta, s, G->gre, G->gim);
    }
    wsync();
    const cd f = {G->fre[r], G->fim[r]};
    cd g, sdg = {0.0, 0.0};
    if (GEN && has_g) {
      g = {G->gre[r], G->gim[r]};
    } else {
      // total-degree start system g_r = x_r^{d_r} - 1
      const int d = deg_r;
      cd xq = {1.0, 0.0};
      for (int e = 1; e < d; ++e) xq = cmul(xq, xc);
      g = cmul(xq, xc);
      g.re -= 1.0;
      sdg = cmul(s, cscale(xq, (double)d));
    }
    const cd hv = cadd(cmul(s, g), cscale(f, te));
    const cd ht = csub(f, cmul(gamma, g));
    b = csel(emode == EV_F, f, csel(emode == EV_H, hv, cd{-ht.re, -ht.im}));
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      const cd v = {Jrr[j], Jri[j]};
      A[j] = csel(j == r, cadd(v, sdg), v);
    }
  }

  // ----------------------------------------------------------------- solve
  // Gauss-Jordan elimination with partial pivoting on [A | b], one row per
  // lane.  Returns this lane's unknown of the solution; sets sing when the
  // matrix has an exactly zero (or NaN) pivot.
  __device__ __forceinline__ cd solve(bool &sing) {
    // [A | b] in one local array (the row state is dead after the solve)
    cd M[NMAX + 1];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) M[j] = A[j];
    M[NMAX] = b;
    bool used = false;
    int pcol = r;
    sing = false;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k < n) {
        double best = -1.0;
        int p = -1;
        if (dpp_groups()) {
          // groups of 2, 4 or 8 aligned lanes: butterfly max over (value,
          // row) in registers (DPP: xor 1, xor 2 within quads, mirror
          // within 8 lanes), no LDS round trip
          best = used ? -1.0 : cabs1(M[k]);
          p = r;
          best = dpp_max_step<0xB1>(best, p);
          if (n >= 4) best = dpp_max_step<0x4E>(best, p);
          if (n >= 8) best = dpp_max_step<0x141>(best, p);
        } else {
          G->cand[r] = used ? -1.0 : cabs1(M[k]);
          wsync();
          double c[NMAX];
#pragma unroll
          for (int q = 0; q < NMAX; ++q) c[q] = G->cand[q];
#pragma unroll
          for (int q = 0; q < NMAX; ++q) {
            const bool take = (q < n) && (c[q] > best);
            best = take ? c[q] : best;
            p = take ? q : p;
          }
        }
        if (!(best > 0.0)) sing = true;
        const bool piv = (r == p);
        if (piv) {
          const cd inv = crecip_nr(M[k]);
#pragma unroll
          for (int j = 0; j <= NMAX; ++j) {
            if (j > k) {
              M[j] = cmul(M[j], inv);
              st(&G->prow[j], M[j]);
            }
          }
          used = true;
          pcol = k;
        }
        wsync();
        cd pr[NMAX + 1];
#pragma unroll
        for (int j = 0; j <= NMAX; ++j)
          if (j > k) pr[j] = ld(&G->prow[j]);
        // rows other than the pivot row: M -= M[k] * pivot row (the pivot
        // row uses a zero multiplier, which leaves it unchanged)
        const cd l = csel(piv, cd{0.0, 0.0}, M[k]);
#pragma unroll
        for (int j = 0; j <= NMAX; ++j)
          if (j > k) M[j] = cfms(M[j], l, pr[j]);
      }
    }
    st(&G->dsol[pcol], M[NMAX]);
    wsync();
    return ld(&G->dsol[r]);
  }

  // ------------------------------------------------------------ start path
  __device__ __forceinline__ void start_path(long long q) {
    qidx = q;
    const long long pid = ids ? ids[q] : id_base + q;
    if (GEN && start) {
      const double2 z = start[pid * n + (r < n ? r : 0)];
      x0 = {z.x, z.y};
    } else {
      const long long kk = (pid / sp->radix[r]) % sp->deg[r];
      const double2 z = a.roots[sp->root_base + sp->root_off[r] + (int)kk];
      x0 = {z.x, z.y};
    }
    mode = M_TRACK;
    t = 0.0;
    h = a.tol.h_init;
    accepts = steps = rejections = newton_its = evals = solves = 0;
  }

  // ------------------------------------------------------------- one step
  // One predictor-corrector attempt for TRACK paths, the final Newton for
  // FINAL paths.  Sets fin_status >= 0 for paths that end here (the endpoint
  // is then x0).  The step runs as a sequence of phases that each make one
  // evaluation (and one solve), so eval() and solve() are instantiated once:
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
    xc = x0;
    int phase = ballot(trk) ? 0 : 4;
    if (phase == 4) iter = fnl;
    for (;;) {
      if (phase == 4 && ballot(iter) == 0) {
        // ---- step control ----
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
        nx = group_max(cmod(x0));
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
        // ---- residual ||f(x0)||_inf of ending paths, classification ----
        res = group_max(cmod(b));
        if (fnl) {
          if (res <= tol.tol_residual && nx <= tol.div_radius) fs = HP_CONVERGED;
          else if (nx > tol.div_radius) fs = HP_DIVERGED;
          else fs = HP_FAILED_NEWTON_T1;
        }
        break;
      }
      bool sing;
      const cd dsl = solve(sing);
      if (phase < 4) {
        // ---- RK4 stage ----
        ok = ok && !sing;
        const double cnext = (phase == 2) ? hs : 0.5 * hs;
        const double wk = (phase == 0 || phase == 3) ? 1.0 : 2.0;
        ks = csel(phase == 0, dsl, cadd(ks, cscale(dsl, wk)));
        xc = csel(phase == 3, cadd(x0, cscale(ks, hs / 6.0)), cadd(x0, cscale(dsl, cnext)));
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
      if (iter && !sing) xc = csub(xc, dsl);
      double md = cmod(dsl), mx = cmod(xc);
      group_max2(md, mx);
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

  // Writes the finished path of this lane's group.
  __device__ __forceinline__ void write_out(int fs, double res) {
    a.endpoints[out_x_base + qidx * n + r] = make_double2(x0.re, x0.im);
    if (r == 0) {
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
  }
};

// ------------------------------------------------------------------------
// Persistent kernel: resident wavefronts loop until every system's queue is
// drained.  A wavefront works on one system at a time and moves on to the
// next system once its queue is empty and its own groups are idle.
// ------------------------------------------------------------------------
template <int NMAX, bool GEN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_persistent(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Tracker<NMAX, GEN> tr(a, smem);
  const int first_sys = blockIdx.x % a.n_systems;
  for (int v = 0; v < a.n_systems; ++v) {
    const int s = (first_sys + v) % a.n_systems;
    tr.load_system(s);
    bool exhausted = false;
    for (;;) {
      // ---- refill idle groups: one atomic per wavefront ----
      const bool idle_leader = tr.leader && tr.mode == M_IDLE;
      const uint64_t m = ballot(idle_leader);
      if (m != 0 && !exhausted) {
        const unsigned cnt = __popcll(m);
        const int first = __builtin_ctzll(m);
        unsigned long long base = 0;
        if (tr.lane == first) base = atomicAdd(&a.qhead[s], (unsigned long long)cnt);
        base = __shfl(base, first);
        const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (idle_leader) {
          const long long q = (long long)base + rank;
          tr.ctl[tr.grp] = q < tr.npaths ? q : -1;
        }
        if ((long long)(base + cnt) >= tr.npaths) exhausted = true;
        wsync();
        if (tr.mode == M_IDLE && tr.grp < tr.ngroups) {
          const long long q = tr.ctl[tr.grp];
          if (q >= 0) tr.start_path(q);
        }
        wsync();
      }
      if (ballot(tr.mode != M_IDLE) == 0) {
        if (exhausted) break;  // this system is drained for this wavefront
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
}

// ------------------------------------------------------------------------
// Plain tracker: one step per launch.  Wavefront b owns queue indices
// [G b, G b + G), G = floor(64 / n), of the single system 0; path state
// lives in HBM between launches.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_plain_init(KArgs a) {
  const DevSys *sd = a.sys;
  const long long q = (long long)blockIdx.x * 64 + threadIdx.x;
  if (q >= sd->n_paths) return;
  const long long P = a.ps.P;
  const long long pid = sd->ids ? sd->ids[q] : sd->id_base + q;
  for (int j = 0; j < sd->n; ++j) {
    if (sd->start) {
      a.ps.x0[j * P + q] = sd->start[pid * sd->n + j];
    } else {
      long long kk = (pid / sd->radix[j]) % sd->deg[j];
      a.ps.x0[j * P + q] = a.roots[sd->root_base + sd->root_off[j] + (int)kk];
    }
  }
  a.ps.t[q] = 0.0;
  a.ps.h[q] = a.tol.h_init;
  a.ps.iv[0 * P + q] = M_TRACK;
  for (int f = 1; f < 8; ++f) a.ps.iv[f * P + q] = 0;
}

template <int NMAX, bool GEN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_plain_step(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Tracker<NMAX, GEN> tr(a, smem);
  tr.load_system(0);
  const long long P = a.ps.P;
  const long long q = (long long)blockIdx.x * tr.ngroups + tr.grp;
  const bool valid = tr.grp < tr.ngroups && q < tr.npaths;
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
    const double2 z = a.ps.x0[tr.r * P + q];
    tr.x0 = {z.x, z.y};
  }
  int fs;
  double res;
  tr.step(fs, res);
  if (fs >= 0) {
    tr.write_out(fs, res);
    tr.mode = M_IDLE;
  }
  if (md != M_IDLE) {
    a.ps.x0[tr.r * P + q] = make_double2(tr.x0.re, tr.x0.im);
    if (tr.r == 0) {
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
  const uint64_t m = ballot(tr.leader && tr.mode != M_IDLE && valid);
  if (tr.lane == 0 && m) atomicAdd(a.ps.active, (unsigned)__popcll(m));
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

template <int NMAX, bool GEN>
static int launch_persistent_t(const KArgs &a, int groups, size_t lds, hipStream_t s) {
  int rc = allow_lds(k_persistent<NMAX, GEN>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_persistent<NMAX, GEN>), dim3(groups), dim3(64), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, bool GEN>
static int launch_plain_t(const KArgs &a, int groups, size_t lds, hipStream_t s) {
  int rc = allow_lds(k_plain_step<NMAX, GEN>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_plain_step<NMAX, GEN>), dim3(groups), dim3(64), lds, s, a);
  return (int)hipGetLastError();
}
template <int NMAX, bool GEN>
static int occupancy_t(size_t lds, int *out) {
  int rc = allow_lds(k_persistent<NMAX, GEN>, lds);
  if (rc) return rc;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_persistent<NMAX, GEN>, 64, lds);
}

#define HP_DISPATCH(NM, GN, CALL)                 \
  switch ((NM) * 2 + ((GN) ? 1 : 0)) {            \
    case 8: return CALL(4, false);                \
    case 9: return CALL(4, true);                 \
    case 16: return CALL(8, false);               \
    case 17: return CALL(8, true);                \
    case 20: return CALL(10, false);              \
    case 21: return CALL(10, true);               \
    case 24: return CALL(12, false);              \
    case 25: return CALL(12, true);               \
    default: return (int)hipErrorInvalidValue;    \
  }

int hp_launch_persistent(int nmax, bool general, const KArgs &a, int groups, size_t lds,
                         void *stream) {
#define CALLP(N, G) launch_persistent_t<N, G>(a, groups, lds, (hipStream_t)stream)
  HP_DISPATCH(nmax, general, CALLP)
#undef CALLP
}

int hp_launch_plain_step(int nmax, bool general, const KArgs &a, int groups, size_t lds,
                         void *stream) {
#define CALLS(N, G) launch_plain_t<N, G>(a, groups, lds, (hipStream_t)stream)
  HP_DISPATCH(nmax, general, CALLS)
#undef CALLS
}

int hp_max_groups_per_cu(int nmax, bool general, size_t lds, int *out) {
#define CALLO(N, G) occupancy_t<N, G>(lds, out)
  HP_DISPATCH(nmax, general, CALLO)
#undef CALLO
}

int hp_launch_plain_init(const KArgs &a, void *stream) {
  const int groups = (int)((a.ps.P + 63) / 64);
  hipLaunchKernelGGL(k_plain_init, dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
