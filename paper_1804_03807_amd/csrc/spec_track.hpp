// One-path-per-lane tracker specialised to one polynomial system.  The
// library writes the system's evaluator S at run time (straight-line code
// with the support, exponents and start-system degrees compiled in; only the
// coefficients are read from memory, through scalar loads) and compiles it
// with this header through hiprtc.  Every index is then a compile-time
// constant, so the Jacobian of a lane's path lives in registers: no atomics,
// and the term loop is plain FP64 arithmetic.  What the registers cannot
// also hold sits in the lane's own LDS slots: its RK4 state, its equation
// values and right-hand side, and its current point during the solve.
//
// S provides
//   static constexpr int N;
//   static constexpr bool kParam;  (the coefficient-parameter form)
//   static void eval(cptr<double2> cf, const cd (&x)[N], double te, cd s,
//                    cd gamma, int emode, cd (&J)[N][N], lds_char *spare);
// which writes J = t J_f + s J_g at (x, te) with s = gamma (1 - te), and
// the right-hand side -H_t (EV_NEG_HT), H (EV_H) or f (EV_F), as the other
// kernels do, to the lane's LDS slots spare + i * 1024.
#pragma once

#include "lane_track.hpp"
#include "reg_lu.hpp"

namespace hp {

// LDS slots per wavefront: RkLds<N> (3N x 1 KB).
template <class S>
struct Spec : LaneTrack<Spec<S>, S::N, RkLds<S::N>> {
  static constexpr int N = S::N;
  // coefficient-parameter form: start points of the launch's paths from
  // memory, coefficient table of (f, g, gamma g - f) per term
  static constexpr bool kStartFromMemory = S::kParam;
  using Base = LaneTrack<Spec<S>, N, RkLds<N>>;
  using Base::a;
  using Base::sp;
  using Base::gamma;
  using Base::xc;

  cptr<double2> coef;  // this system's term coefficients, in packed order
  cd J[N][N];
  cd b[N];

  // lds: the wavefront's RkLds<N>::kBytes
  __device__ Spec(const KArgs &args, lds_char *lds)
      : Base(args, true, lds + (threadIdx.x & 63) * 16) {}

  __device__ __forceinline__ void load_system(int s) {
    this->load_common(s);
    if constexpr (S::kParam) coef = as_const(a.pcoef) + 3 * (long long)sp->term_base;
    else coef = as_const(a.tcoef) + sp->term_base;
  }

  // [J | rhs]: J in registers, the right-hand side in the lane's spare LDS
  // slots (the evaluator leaves each equation's value there after its last
  // term, then its right-hand side)
  __device__ __forceinline__ void eval(int emode, double te) {
    S::eval(coef, xc, te, cscale(gamma, 1.0 - te), gamma, emode, J, this->rk.spare_base());
    // Hand J over to the solve as opaque register values: otherwise the
    // compiler interleaves the evaluation with the elimination and needs
    // far more registers than either (scratch spills from n = 7 on).
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) asm volatile("" : "+v"(J[i][j].re), "+v"(J[i][j].im));
    }
    asm volatile("" ::: "memory");
  }

  // right-hand side from LDS; the current point waits in LDS during the
  // elimination
  __device__ __forceinline__ void solve(cd dx[N], bool &sing, bool live) {
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = this->rk.spare(i);
    this->rk.park(xc);
    reg_lu_solve<N, (N <= 8), false>(J, b, dx, sing, live);
    this->rk.unpark(xc);
  }

  __device__ __forceinline__ double residual() const {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) r = nmax(r, cmod(this->rk.spare(i)));
    return r;
  }
};

}  // namespace hp
