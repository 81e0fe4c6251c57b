// Per-lane path tracking shared by the one-path-per-lane kernels: the path
// state, start points, the predictor-corrector step with its step-size
// control and end game, the output record, and the persistent and plain
// kernel bodies.  A tracker D derives from LaneTrack<D, N> and supplies
//   void eval(int emode, double te);    [J_x(xc, te) | rhs], see EvalMode
//   void solve(cd dx[N], bool &sing, bool live);
//                                       J dx = rhs; lanes with live false
//                                       discard dx and sing
//   double residual() const;            max_i |rhs_i| after eval(EV_F, 1)
// Compiled by hipcc into the library and by hiprtc into the kernels that
// are specialised to one system at run time.
#pragma once

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

// Where a lane keeps the accepted point x0 and the RK4 accumulator ks of its
// path: registers, or (RkLds) its own LDS slots, for trackers whose
// registers are taken by the Jacobian.
template <int N>
struct RkRegs {
  cd x0v[N], ksv[N];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < N; ++i) x0v[i] = ksv[i] = {0.0, 0.0};
  }
  __device__ __forceinline__ cd x0(int i) const { return x0v[i]; }
  __device__ __forceinline__ void set_x0(int i, cd v) { x0v[i] = v; }
  __device__ __forceinline__ cd ks(int i) const { return ksv[i]; }
  __device__ __forceinline__ void set_ks(int i, cd v) { ksv[i] = v; }
};
// Lane-major: slot e of the wavefront is 64 x 16 bytes, lane l's value at
// byte e * 1024 + l * 16 (every access is one contiguous block); x0 in slots
// 0..N-1, ks in slots N..2N-1, and slots 2N..3N-1 park the current point
// while the elimination needs the registers (park / unpark).
template <int N>
struct RkLds {
  static constexpr int kBytes = 3 * N * 64 * 16;  // per wavefront
  lds_char *p;  // this lane's value in slot 0
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2 * N; ++i) stl(p + i * 1024, {0.0, 0.0});
  }
  __device__ __forceinline__ cd x0(int i) const { return ldl(p + i * 1024); }
  __device__ __forceinline__ void set_x0(int i, cd v) { stl(p + i * 1024, v); }
  __device__ __forceinline__ cd ks(int i) const { return ldl(p + (N + i) * 1024); }
  __device__ __forceinline__ void set_ks(int i, cd v) { stl(p + (N + i) * 1024, v); }
  // slot 2N + i (the parking slots) one value at a time
  __device__ __forceinline__ lds_char *spare_base() const { return p + 2 * N * 1024; }
  __device__ __forceinline__ cd spare(int i) const { return ldl(p + (2 * N + i) * 1024); }
  __device__ __forceinline__ void set_spare(int i, cd v) { stl(p + (2 * N + i) * 1024, v); }
  // x to LDS and back; the memory barriers keep the compiler from carrying
  // the values in registers across (it must reload them)
  __device__ __forceinline__ void park(const cd (&x)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) stl(p + (2 * N + i) * 1024, x[i]);
    asm volatile("" ::: "memory");
  }
  __device__ __forceinline__ void unpark(cd (&x)[N]) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = ldl(p + (2 * N + i) * 1024);
  }
};

// N: the number of unknowns, exact (a system of another n runs on another
// instantiation), so every loop over unknowns is unrolled without guards.
//
// Method (paper: Section 1 and the end of Section 2.1 for independent paths
// and dynamic load balancing).  H(x,t) = gamma (1-t) g(x) + t f(x) with the
// total-degree start system g_i = x_i^{d_i} - 1; one RK4 predictor step on
// the path's differential equation and Newton corrector iterations form a
// step; step control and the end game are those of the library's
// documented reading (halving on a rejection, doubling after three
// accepts, final Newton and residual test at t = 1).
template <class D, int N, class Rk = RkRegs<N>>
struct LaneTrack {
  static constexpr int NMAX = N;
  static constexpr int n = N;
  // a tracker whose paths start at points in memory (DevSys::start) declares
  // kStartFromMemory = true; the others decode start points from path ids
  static constexpr bool kStartFromMemory = false;

  const KArgs &a;
  const int lane;
  const bool slot;  // lane holds paths
  // ---- current system (wave-uniform) ----
  cptr<DevSys> sp;
  int deg[N];
  cd gamma;
  long long npaths, out_path_base, out_x_base, id_base;
  const long long *ids;
  // ---- path state ----
  int mode, accepts, steps, rejections, newton_its, evals, solves;
  long long qidx;
  double t, h;
  cd xc[N];  // current point
  Rk rk;     // accepted point x0 and RK4 accumulator ks

  // rk_lds: the lane's slot-0 address for RkLds (unused for RkRegs)
  __device__ LaneTrack(const KArgs &args, bool holds_paths, lds_char *rk_lds = nullptr)
      : a(args), lane(threadIdx.x & 63), slot(holds_paths) {
    mode = M_IDLE;
    t = h = 0.0;
    qidx = 0;
    accepts = steps = rejections = newton_its = evals = solves = 0;
    if constexpr (!__is_same(Rk, RkRegs<N>)) rk.p = rk_lds;
    rk.init();
#pragma unroll
    for (int i = 0; i < N; ++i) xc[i] = {0.0, 0.0};
  }

  __device__ __forceinline__ D &self() { return *static_cast<D *>(this); }

  // System fields every lane tracker needs.
  __device__ __forceinline__ void load_common(int s) {
    sp = as_const(a.sys) + s;
#pragma unroll
    for (int i = 0; i < N; ++i) deg[i] = sp->deg[i];
    gamma = {sp->gre, sp->gim};
    npaths = sp->n_paths;
    out_path_base = sp->out_path_base;
    out_x_base = sp->out_x_base;
    ids = (const long long *)sp->ids;
    id_base = sp->id_base;
  }

  // output slot of queue index q
  __device__ __forceinline__ long long slot_of(long long q) const {
    const long long *sl = (const long long *)sp->slots;
    return sl ? sl[q] : q;
  }

  // A path suspended at the end of an earlier launch resumes from its slot:
  // accepted point, t, h and counters as suspend() left them.
  __device__ __forceinline__ bool resume(long long q) {
    const long long o = out_path_base + slot_of(q);
    const int st = a.status[o];
    if (st != kSuspendedTrack && st != kSuspendedFinal) return false;
    const double2 *e = a.endpoints + out_x_base + slot_of(q) * n;
#pragma unroll
    for (int i = 0; i < N; ++i) rk.set_x0(i, {e[i].x, e[i].y});
    const hp_path_stats *s = a.stats + o;
    steps = s->steps;
    rejections = s->rejections;
    newton_its = s->newton_iters;
    evals = s->evals;
    solves = s->solves;
    accepts = s->pad;
    t = s->t_final;
    h = s->residual;
    mode = (st == kSuspendedFinal) ? M_FINAL : M_TRACK;
    return true;
  }

  // The step budget of the launch is spent: the path's state goes to its
  // slot (endpoint = accepted point; stats hold t, h, counters).
  __device__ __forceinline__ void suspend() {
    const long long so = slot_of(qidx);
    double2 *e = a.endpoints + out_x_base + so * n;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const cd x = rk.x0(i);
      e[i] = make_double2(x.re, x.im);
    }
    hp_path_stats *s = a.stats + out_path_base + so;
    s->steps = steps;
    s->rejections = rejections;
    s->newton_iters = newton_its;
    s->evals = evals;
    s->solves = solves;
    s->pad = accepts;
    s->t_final = t;
    s->residual = h;
    a.status[out_path_base + so] = (mode == M_FINAL) ? kSuspendedFinal : kSuspendedTrack;
  }

  // ------------------------------------------------------------ start path
  // Path id -> start point of the total-degree start system: digit i of the
  // id in the mixed radix (d_0, d_1, ...) picks the root of unity of x_i.
  // Sliced: the launch may find suspended paths in its queue (serving).
  template <bool Sliced>
  __device__ __forceinline__ void start_path(long long q) {
    qidx = q;
    if constexpr (Sliced) {
      if (resume(q)) return;
    }
    const long long pid = ids ? ids[q] : id_base + q;
    if constexpr (D::kStartFromMemory) {
      const double2 *st = sp->start + pid * N;
#pragma unroll
      for (int i = 0; i < N; ++i) rk.set_x0(i, {st[i].x, st[i].y});
    } else {
      cptr<double> roots = as_const((const double *)a.roots) + 2 * sp->root_base;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const long long kk = (pid / sp->radix[i]) % deg[i];
        const int ri = sp->root_off[i] + (int)kk;
        rk.set_x0(i, {roots[2 * ri], roots[2 * ri + 1]});
      }
    }
    mode = M_TRACK;
    t = 0.0;
    h = a.tol.h_init;
    accepts = steps = rejections = newton_its = evals = solves = 0;
  }

  __device__ __forceinline__ static double vmax_mod(const cd v[N]) {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) m = nmax(m, cmod(v[i]));
    return m;
  }
  __device__ __forceinline__ double x0_max_mod() const {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) m = nmax(m, cmod(rk.x0(i)));
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
    for (int i = 0; i < N; ++i) xc[i] = rk.x0(i);
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
            for (int i = 0; i < N; ++i) rk.set_x0(i, xc[i]);
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
          for (int i = 0; i < N; ++i) rk.set_x0(i, xc[i]);
        }
        nx = x0_max_mod();
        if (trk) {
          if (nx > tol.div_radius) fs = HP_DIVERGED;
          else if (t >= 1.0) mode = M_FINAL;
          else if (h < tol.h_min) fs = HP_FAILED_MINSTEP;
          else if (steps > tol.max_steps) fs = HP_FAILED_MAXSTEPS;
        }
        if (ballot(fs >= 0 || fnl) == 0) break;
        phase = 5;
#pragma unroll
        for (int i = 0; i < N; ++i) xc[i] = rk.x0(i);
      }
      const double te = (phase == 0) ? (trk ? t : 1.0)
                      : (phase == 1 || phase == 2) ? (trk ? th : 1.0)
                      : (phase == 3 || phase == 4) ? tn : 1.0;
      self().eval(phase < 4 ? EV_NEG_HT : (phase == 4 ? EV_H : EV_F), te);
      if (phase == 5) {
        // ---- residual ||f(x0)||_inf of ending paths, classification ----
        res = self().residual();
        if (fnl) {
          if (res <= tol.tol_residual && nx <= tol.div_radius) fs = HP_CONVERGED;
          else if (nx > tol.div_radius) fs = HP_DIVERGED;
          else fs = HP_FAILED_NEWTON_T1;
        }
        break;
      }
      bool sing;
      cd dsl[N];
      // the RK4 stages serve the tracking lanes, a Newton iteration the
      // lanes still iterating; the other lanes run along and discard dx
      self().solve(dsl, sing, phase < 4 ? trk : iter);
      if (phase < 4) {
        // ---- RK4 stage ----
        ok = ok && !sing;
        const double cnext = (phase == 2) ? hs : 0.5 * hs;
        const double wk = (phase == 0 || phase == 3) ? 1.0 : 2.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const cd k = csel(phase == 0, dsl[i], cadd(rk.ks(i), cscale(dsl[i], wk)));
          const cd x = rk.x0(i);
          rk.set_ks(i, k);
          xc[i] = csel(phase == 3, cadd(x, cscale(k, hs / 6.0)), cadd(x, cscale(dsl[i], cnext)));
        }
        if (phase == 3) {
          if (trk) {
            evals += 4;
            solves += 4;
          }
          if (fnl) {
#pragma unroll
            for (int i = 0; i < N; ++i) xc[i] = rk.x0(i);
          }
          iter = (trk && ok) || fnl;
        }
        ++phase;
        continue;
      }
      // ---- Newton iteration: x -= dx ----
      if (iter && !sing) {
#pragma unroll
        for (int i = 0; i < N; ++i) xc[i] = csub(xc[i], dsl[i]);
      }
      const double md = vmax_mod(dsl), mx = vmax_mod(xc);
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

  // Sliced: queue indices map to slots (serving)
  template <bool Sliced = false>
  __device__ __forceinline__ void write_out(int fs, double res) {
    long long so = qidx;
    if constexpr (Sliced) so = slot_of(qidx);
    double2 *e = a.endpoints + out_x_base + so * n;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const cd x = rk.x0(i);
      e[i] = make_double2(x.re, x.im);
    }
    const long long o = out_path_base + so;
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
// Persistent body: resident wavefronts loop until every system's queue is
// drained; a wavefront moves to the next system once its queue is empty and
// its own lanes are idle.  Idle lanes are refilled from one device queue
// head per system with one atomicAdd per wavefront (ballot, popcount,
// mbcnt), in place of the work crew's guarded next-job pointer (Section 1).
// ------------------------------------------------------------------------
// Drains system s's queue: tracks its paths until the queue is empty and
// this wavefront's lanes are idle.  Sliced (serving): queue entries may be
// paths suspended by an earlier launch, which resume from their slots, and
// once the wavefront has taken a.step_budget > 0 steps in this launch
// (counted in wave_steps across the systems it visits) its paths in flight
// are suspended to their slots and it returns true.
template <bool Sliced, class T>
__device__ __forceinline__ bool lane_drain(const KArgs &a, T &tr, int s, int &wave_steps) {
  tr.load_system(s);
  bool exhausted = false;
  for (;;) {
    if constexpr (Sliced) {
      if (a.step_budget > 0 && wave_steps >= a.step_budget) {
        if (tr.slot && tr.mode != M_IDLE) {
          tr.suspend();
          tr.mode = M_IDLE;
        }
        return true;
      }
    }
    // ---- refill idle lanes: one atomic per wavefront (lanes past the
    // launch's paths per wavefront stay idle) ----
    const bool idle = tr.slot && tr.mode == M_IDLE && lane_holds_path(a);
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
        if (q < tr.npaths) tr.template start_path<Sliced>(q);
      }
      if ((long long)(qb + cnt) >= tr.npaths) exhausted = true;
    }
    if (ballot(tr.mode != M_IDLE) == 0) {
      if (exhausted) break;  // this system is drained for this wavefront
      continue;
    }
    // lanes that hold no path slot sit out the step
    if (tr.slot) {
      int fs;
      double res;
      tr.step(fs, res);
      if (fs >= 0) {
        tr.template write_out<Sliced>(fs, res);
        tr.mode = M_IDLE;
      }
    }
    if constexpr (Sliced) ++wave_steps;
  }
  return false;
}

template <bool Sliced = false, class T>
__device__ __forceinline__ void lane_persistent(const KArgs &a, T &tr) {
  const int first_sys = blockIdx.x % a.n_systems;
  int wave_steps = 0;
  for (int v = 0; v < a.n_systems; ++v)
    if (lane_drain<Sliced>(a, tr, (first_sys + v) % a.n_systems, wave_steps)) return;
}

// ------------------------------------------------------------------------
// Plain body: one step per launch.  Wavefront b owns queue indices
// [PW b, PW b + PW) of system 0; path state lives in HBM between launches
// (initialised by k_plain_init).
// ------------------------------------------------------------------------
template <class T, int PW>
__device__ __forceinline__ void lane_plain(const KArgs &a, T &tr) {
  constexpr int N = T::NMAX;
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
      tr.rk.set_x0(i, {z.x, z.y});
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
    for (int i = 0; i < N; ++i) {
      const cd x = tr.rk.x0(i);
      a.ps.x0[i * P + q] = make_double2(x.re, x.im);
    }
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
