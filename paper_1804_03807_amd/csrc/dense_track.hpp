// Dense one-path-per-lane tracker for gfx950 (CDNA4), complex FP64:
// systems of n <= kDenseMaxN unknowns whose equations have total degree at
// most 3, stored as full coefficient tables (every monomial of the degree,
// zero where absent; layout in hp_internal.hpp).
//
// Evaluation.  With the loops over variables unrolled for the compile-time
// n, an equation is evaluated in nested (Horner) form and its gradient in
// reverse mode over the same form (dense_eval.hpp): two complex
// multiply-adds per cubic monomial, every index a compile-time constant, so
// the Jacobian row is a register array and the whole Jacobian stays in
// registers for the register LU, as in the kernels specialised at run time;
// the right-hand side, the RK4 state and (during the solve) the current
// point sit in the lane's own LDS slots.
// The partial derivatives are scaled by t and the start system
// g_i = x_i^{d_i} - 1 is added as in the other kernels (paper: Section 1;
// the end of Section 2.1 for independent paths).
//
// Kernels: k_dense (dense.hip) tracks every system of a launch with
// n <= kDenseMaxN, dispatching per system on n; k_dense_n<11> and k_dense_n<12>
// (dense11.hip, dense12.hip: translation units of their own, so that the
// largest instantiations compile in parallel) track systems of exactly that
// n.
#pragma once

#include "dense_eval.hpp"
#include "lane_track.hpp"
#include "reg_lu.hpp"

namespace hp {

template <int N>
struct Dense : LaneTrack<Dense<N>, N, RkLds<N>> {
  using Base = LaneTrack<Dense<N>, N, RkLds<N>>;
  using Base::a;
  using Base::sp;
  using Base::gamma;
  using Base::xc;
  using Base::deg;

  cptr<double> dc;  // this system's dense table, (re, im) pairs
  int off[N];       // first coefficient of equation i
  cd J[N][N];
  cd b[N];

  // lds: at least RkLds<N>::kBytes
  __device__ Dense(const KArgs &args, lds_char *lds)
      : Base(args, true, lds + (threadIdx.x & 63) * 16) {}

  __device__ __forceinline__ void load_system(int s) {
    this->load_common(s);
    dc = as_const((const double *)a.dcoef) + 2 * (long long)sp->dense_base;
#pragma unroll
    for (int i = 0; i < N; ++i) off[i] = sp->dense_off[i];
  }

  // Equation of total degree D whose table starts at c at the current point:
  // returns its value and writes its gradient to g.
  template <int D>
  __device__ __forceinline__ cd equation(cptr<double> c, cd (&g)[N]) const {
    return dense_equation<N, D>(c, xc, g);
  }

  // [J_x(xc, te) | rhs]: J = t J_f + s J_g, rhs = -H_t, H or f (EvalMode).
  __device__ __forceinline__ void eval(int emode, double te) {
    const cd s = cscale(gamma, 1.0 - te);
    sfor<0, N>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      cd g[N];
      const cptr<double> c = dc + 2 * off[i];
      const int d = deg[i];
      cd f;
      if (d >= 3) f = equation<3>(c, g);
      else if (d == 2) f = equation<2>(c, g);
      else f = equation<1>(c, g);
#pragma unroll
      for (int j = 0; j < N; ++j) J[i][j] = cscale(g[j], te);
      // start system x_i^{d_i} - 1 (d_i <= 3)
      cd xq = (d >= 2) ? xc[i] : cd{1.0, 0.0};
      if (d >= 3) xq = cmul(xq, xc[i]);
      cd gs = cmul(xq, xc[i]);
      gs.re -= 1.0;
      J[i][i] = cadd(J[i][i], cmul(s, cscale(xq, (double)d)));
      const cd hv = cadd(cmul(s, gs), cscale(f, te));
      const cd mht = csub(cmul(gamma, gs), f);
      // the right-hand side waits in the lane's spare LDS slots until the
      // solve, leaving the registers to the Jacobian rows
      this->rk.set_spare(i, csel(emode == EV_F, f, csel(emode == EV_H, hv, mht)));
      // the finished row as opaque values: equations are not interleaved
#pragma unroll
      for (int j = 0; j < N; ++j) asm volatile("" : "+v"(J[i][j].re), "+v"(J[i][j].im));
    });
    asm volatile("" ::: "memory");
  }

  // right-hand side from LDS; the current point waits in LDS during the
  // elimination
  __device__ __forceinline__ void solve(cd dx[N], bool &sing, bool live) {
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = this->rk.spare(i);
    this->rk.park(xc);
    // row blocks pay in the kernel for n <= 10; the kernels of n = 11, 12
    // (mostly spills either way) run faster without them
    reg_lu_solve<N, true, (N <= kDenseMaxN)>(J, b, dx, sing, live);
    this->rk.unpark(xc);
  }

  __device__ __forceinline__ double residual() const {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) r = nmax(r, cmod(this->rk.spare(i)));
    return r;
  }
};

// true when the launch's step budget stopped the wavefront (Sliced)
template <int N, bool Sliced>
__device__ __forceinline__ bool dense_drain(const KArgs &a, int s, lds_char *rk, int &wave_steps) {
  Dense<N> tr(a, rk);
  return lane_drain<Sliced>(a, tr, s, wave_steps);
}

// Persistent kernel over every system of the launch (n <= kDenseMaxN, mixed
// n in one launch): a wavefront drains the systems' refill queues one after
// another and runs the tracker instantiated for each system's n
// (wave-uniform).  Sliced: the serving form (suspend and resume, see
// lane_drain).
template <bool Sliced>
__global__ void __launch_bounds__(64) k_dense(KArgs a) {
  __shared__ __align__(16) char rk[RkLds<kDenseMaxN>::kBytes];
  lds_char *lds = (lds_char *)rk;
  const int first_sys = blockIdx.x % a.n_systems;
  int wave_steps = 0;
  for (int v = 0; v < a.n_systems; ++v) {
    const int s = (first_sys + v) % a.n_systems;
    bool stop = false;
    switch (as_const(a.sys)[s].n) {
      case 1: stop = dense_drain<1, Sliced>(a, s, lds, wave_steps); break;
      case 2: stop = dense_drain<2, Sliced>(a, s, lds, wave_steps); break;
      case 3: stop = dense_drain<3, Sliced>(a, s, lds, wave_steps); break;
      case 4: stop = dense_drain<4, Sliced>(a, s, lds, wave_steps); break;
      case 5: stop = dense_drain<5, Sliced>(a, s, lds, wave_steps); break;
      case 6: stop = dense_drain<6, Sliced>(a, s, lds, wave_steps); break;
      case 7: stop = dense_drain<7, Sliced>(a, s, lds, wave_steps); break;
      case 8: stop = dense_drain<8, Sliced>(a, s, lds, wave_steps); break;
      case 9: stop = dense_drain<9, Sliced>(a, s, lds, wave_steps); break;
      case 10: stop = dense_drain<10, Sliced>(a, s, lds, wave_steps); break;
      default: break;  // the host admits n <= kDenseMaxN only
    }
    if (stop) return;  // the step budget is spent
  }
}

// The same for systems of exactly n = N (11, 12), one instantiation per
// translation unit so that they compile side by side.
template <int N, bool Sliced>
__global__ void __launch_bounds__(64) k_dense_n(KArgs a) {
  __shared__ __align__(16) char rk[RkLds<N>::kBytes];
  const int first_sys = blockIdx.x % a.n_systems;
  int wave_steps = 0;
  for (int v = 0; v < a.n_systems; ++v)
    if (dense_drain<N, Sliced>(a, (first_sys + v) % a.n_systems, (lds_char *)rk, wave_steps)) return;
}

// Launch and occupancy of one instantiation (hipError_t values).
template <class K>
int dense_launch(K kernel, const KArgs &a, int groups, void *stream) {
  hipLaunchKernelGGL(kernel, dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
template <class K>
int dense_per_cu(K kernel, int *out) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, kernel, 64, 0);
}

}  // namespace hp
