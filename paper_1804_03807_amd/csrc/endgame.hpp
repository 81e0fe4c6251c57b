// End game at t = 1 for gfx950, run after the tracking kernels: Newton
// refinement of each endpoint with f evaluated in double-double arithmetic,
// then the residual test at the nearest double of the refined point, again
// with f in double-double.
//
// Why.  The tracking kernels end a path with a double-precision Newton at
// t = 1, whose endpoint and residual depend on the order of the arithmetic
// that led there: two correct implementations can put a root whose residual
// sits at the rounding floor on opposite sides of the absolute residual
// gate.  Refined in double-double, the endpoint is the double nearest to the
// root, and the residual is that of this double, computed accurately, so
// the finite / not-finite split of the endpoints (paper: Section 3.1,
// Figure 3, solutions at infinity and finite ones) no longer depends on
// evaluation order.  Double-double arithmetic is the paper's means to more
// accurate results (Section 1; Section 5.1 times the blackbox solver in
// double-double precision).
//
// Mapping.  One path per lane, 64 per wavefront, one instantiation per n so
// that the point, the residual and the Jacobian are register arrays; the
// terms come in equation order through scalar loads (every lane of a block
// works on the same system), so the exponents of a term are wave-uniform
// and every variable index is a compile-time constant.  Paths that the
// dense kernels tracked take the dense form instead: f from the systems'
// dense coefficient tables in nested form, in double-double, and J_f by the
// dense kernels' reverse-mode sweep (one complex multiply-add per monomial
// for f, where the term form multiplies out every power).
//
// Per path that the tracker ended CONVERGED or FAILED_NEWTON_T1 with a
// finite endpoint x of ||x||_inf <= div_radius:
//   kRefine times: r = f(x) in double-double rounded to double, J = J_f at
//   the double nearest to x, solve J d = r in double, x <- x - d in
//   double-double (stop on a zero pivot or a non-finite d);
//   x <- nearest double; residual ||f(x)||_inf with f in double-double;
//   CONVERGED if residual <= tol_residual and ||x||_inf <= div_radius, else
//   DIVERGED if ||x||_inf > div_radius, else FAILED_NEWTON_T1.
#pragma once

#include <hip/hip_runtime.h>

#include "dense_eval.hpp"
#include "hp_device.hpp"
#include "hp_internal.hpp"
#include "lane_track.hpp"
#include "reg_lu.hpp"

#include "dd_arith.hpp"  // switches floating-point contraction off for the including file

namespace hp {
namespace {

constexpr int kRefine = 2;  // double-double Newton iterations

// ---- terms ---------------------------------------------------------------
// The end game's copy of a term: coefficient, and the exponent of variable j
// in bits 4j .. 4j+3 of a 64-bit word (exponents are at most 15), so every
// variable index below is a compile-time constant and the point stays in
// registers.
template <int N>
struct Endgame {
  cptr<double> coef;   // this system's equation-ordered terms (re, im)
  cptr<uint32_t> ex;   // 4 words per term: exponent nibbles (low, high), 0, 0
  cptr<int32_t> ep;    // equation i owns terms ep[i] .. ep[i+1]-1

  __device__ __forceinline__ void init(const KArgs &a, cptr<DevSys> sp) {
    coef = as_const((const double *)a.tcoef) + 2 * (long long)sp->eg_base;
    ex = as_const((const uint32_t *)a.tmeta) + 4 * (long long)sp->eg_base;
    ep = as_const(sp->eg_ptr);
  }

  __device__ __forceinline__ uint64_t exps(int t) const {
    return (uint64_t)ex[4 * t] | ((uint64_t)ex[4 * t + 1] << 32);
  }
  __device__ __forceinline__ static int ex_of(uint64_t w, int j) { return (int)((w >> (4 * j)) & 15); }

  // f_i at the double-double point x, rounded to the nearest double
  __device__ __forceinline__ cd f_dd(int i, const cdd (&x)[N]) const {
    cdd acc = {{0.0, 0.0}, {0.0, 0.0}};
    for (int t = ep[i]; t < ep[i + 1]; ++t) {
      const uint64_t w = exps(t);
      cdd v = to_cdd({coef[2 * t], coef[2 * t + 1]});
      sfor<0, N>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        for (int e = ex_of(w, j); e > 0; --e) v = cddmul(v, x[j]);
      });
      acc = cddadd(acc, v);
    }
    return round_cd(acc);
  }

  // row i of J_f at the double point x.  The partial derivative of a term by
  // x_m is its coefficient times e_m x_m^(e_m - 1) times the powers of the
  // variables before m (prefix products) and after m (suffix products).
  __device__ __forceinline__ void jac_row(int i, const cd (&x)[N], cd (&row)[N]) const {
    sfor<0, N>([&](auto jj) { row[decltype(jj)::value] = {0.0, 0.0}; });
    for (int t = ep[i]; t < ep[i + 1]; ++t) {
      const uint64_t w = exps(t);
      cd pw[N], pre[N];
      cd run = {coef[2 * t], coef[2 * t + 1]};
      sfor<0, N>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        pre[j] = run;  // coefficient times the powers of x_0 .. x_{j-1}
        cd p = {1.0, 0.0};
        for (int e = ex_of(w, j); e > 0; --e) p = cmul(p, x[j]);
        pw[j] = p;
        if (ex_of(w, j) > 0) run = cmul(run, p);
      });
      cd suf = {1.0, 0.0};  // powers of x_{m+1} .. x_{N-1}
      sfor<0, N>([&](auto mm) {
        constexpr int m = N - 1 - decltype(mm)::value;
        const int em = ex_of(w, m);
        if (em > 0) {
          cd q = {1.0, 0.0};
          for (int e = em - 1; e > 0; --e) q = cmul(q, x[m]);
          row[m] = cadd(row[m], cmul(cmul(pre[m], cscale(q, (double)em)), suf));
          suf = cmul(suf, pw[m]);
        }
      });
    }
  }
};

// complex double-double times complex double
__device__ __forceinline__ cdd cddmul_cd(cdd a, cd b) {
  return {ddadd(ddmul_d(a.re, b.re), ddneg(ddmul_d(a.im, b.im))),
          ddadd(ddmul_d(a.re, b.im), ddmul_d(a.im, b.re))};
}

// The same interface for systems with dense coefficient tables (the dense
// kernels' systems, total degree <= 3): f_i in double-double in the nested
// form S_ab = q_ab + sum_c k_abc x_c, T_a = l_a + sum_b x_b S_ab,
// f = c + sum_a x_a T_a, and row i of J_f from the dense kernels' sweep.
template <int N>
struct DenseEndgame {
  cptr<double> dc;  // this system's dense table, (re, im) pairs
  cptr<DevSys> sp;

  __device__ __forceinline__ void init(const KArgs &a, cptr<DevSys> s) {
    sp = s;
    dc = as_const((const double *)a.dcoef) + 2 * (long long)s->dense_base;
  }

  template <int D>
  __device__ __forceinline__ static cdd value(cptr<double> c, const cdd (&x)[N]) {
    using T = DenseTable<N>;
    cdd f = to_cdd(T::coef(c, 0));
    sfor<0, N>([&](auto ia) {
      constexpr int va = decltype(ia)::value;
      cdd Ta = to_cdd(T::coef(c, 1 + va));
      if constexpr (D >= 2) {
        sfor<va, N>([&](auto ib) {
          constexpr int vb = decltype(ib)::value;
          cdd S = to_cdd(T::coef(c, T::quad_at(va, vb)));
          if constexpr (D >= 3) {
            sfor<vb, N>([&](auto ic) {
              constexpr int vc = decltype(ic)::value;
              S = cddadd(S, cddmul_cd(x[vc], T::coef(c, T::cubic_at(va, vb, vc))));
            });
          }
          Ta = cddadd(Ta, cddmul(x[vb], S));
        });
      }
      f = cddadd(f, cddmul(x[va], Ta));
    });
    return f;
  }

  // f_i at the double-double point x, rounded to the nearest double
  __device__ __forceinline__ cd f_dd(int i, const cdd (&x)[N]) const {
    const cptr<double> c = dc + 2 * sp->dense_off[i];
    const int d = sp->deg[i];
    if (d >= 3) return round_cd(value<3>(c, x));
    if (d == 2) return round_cd(value<2>(c, x));
    return round_cd(value<1>(c, x));
  }

  // row i of J_f at the double point x
  __device__ __forceinline__ void jac_row(int i, const cd (&x)[N], cd (&row)[N]) const {
    const cptr<double> c = dc + 2 * sp->dense_off[i];
    const int d = sp->deg[i];
    if (d >= 3) dense_equation<N, 3>(c, x, row);
    else if (d == 2) dense_equation<N, 2>(c, x, row);
    else dense_equation<N, 1>(c, x, row);
  }
};

template <int N>
__device__ __forceinline__ double max_mod(const cd (&v)[N]) {
  double m = 0.0;
  sfor<0, N>([&](auto i) { m = nmax(m, cmod(v[decltype(i)::value])); });
  return m;
}

// E: Endgame<N> (terms) or DenseEndgame<N> (dense tables)
template <int N, class E>
__global__ void __launch_bounds__(64) k_endgame(KArgs a, const int2 *blk) {
  const int lane = threadIdx.x & 63;
  int s = 0;
  long long q = (long long)blockIdx.x * 64 + lane;
  if (blk) {
    const int2 b = blk[blockIdx.x];
    s = b.x;
    q = (long long)b.y + lane;
  }
  cptr<DevSys> sp = as_const(a.sys) + s;
  if (a.eg_list) {
    if (q >= (long long)a.eg_count[s]) return;
    q = a.eg_list[sp->eg_list_base + q];
  }
  if (q >= sp->n_paths) return;
  // output slot of queue index q (serving keeps paths in slots of an arena)
  const long long *slots = (const long long *)sp->slots;
  const long long so = slots ? slots[q] : q;
  const long long o = sp->out_path_base + so;
  const int st0 = a.status[o];
  if (st0 != HP_CONVERGED && st0 != HP_FAILED_NEWTON_T1) return;
  double2 *xe = a.endpoints + sp->out_x_base + so * N;
  cd x[N];
  bool finite = true;
  sfor<0, N>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const double2 z = xe[i];
    x[i] = {z.x, z.y};
    finite = finite && (fabs(z.x) < __builtin_inf()) && (fabs(z.y) < __builtin_inf());
  });
  const double div = a.tol.div_radius;
  if (!finite || !(max_mod<N>(x) <= div)) return;

  E ev;
  ev.init(a, sp);

  cdd xv[N];
  sfor<0, N>([&](auto i) { xv[decltype(i)::value] = to_cdd(x[decltype(i)::value]); });
  for (int it = 0; it < kRefine; ++it) {
    cd xh[N], r[N], d[N];
    cd J[N][N];
    sfor<0, N>([&](auto i) { xh[decltype(i)::value] = round_cd(xv[decltype(i)::value]); });
    // equations in a run-time loop (one copy of the term code); rows land
    // in their registers by a select on the equation index
#pragma nounroll
    for (int i = 0; i < N; ++i) {
      const cd fi = ev.f_dd(i, xv);
      cd row[N];
      ev.jac_row(i, xh, row);
      sfor<0, N>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if (i == k) {
          r[k] = fi;
          sfor<0, N>([&](auto jj) { J[k][decltype(jj)::value] = row[decltype(jj)::value]; });
        }
      });
    }
    bool sing = false;
    reg_lu_solve<N, false, false>(J, r, d, sing, true);
    bool ok = !sing;
    sfor<0, N>([&](auto i) {
      const cd di = d[decltype(i)::value];
      ok = ok && (fabs(di.re) < __builtin_inf()) && (fabs(di.im) < __builtin_inf());
    });
    if (!ok) break;
    sfor<0, N>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      xv[i] = cddadd(xv[i], to_cdd({-d[i].re, -d[i].im}));
    });
  }
  cdd xr[N];
  sfor<0, N>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    x[i] = round_cd(xv[i]);
    xr[i] = to_cdd(x[i]);
  });
  const double nx = max_mod<N>(x);
  double res = 0.0;
#pragma nounroll
  for (int i = 0; i < N; ++i) res = nmax(res, cmod(ev.f_dd(i, xr)));
  const int st = (res <= a.tol.tol_residual && nx <= div) ? HP_CONVERGED
                 : (nx > div)                            ? HP_DIVERGED
                                                         : HP_FAILED_NEWTON_T1;
  sfor<0, N>([&](auto i) {
    xe[decltype(i)::value] = make_double2(x[decltype(i)::value].re, x[decltype(i)::value].im);
  });
  a.status[o] = st;
  if (a.stats) a.stats[o].residual = res;
}

template <int N, class E>
int endgame_launch(const KArgs &a, const int2 *blk, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_endgame<N, E>), dim3((unsigned)blocks), dim3(64), 0, s, a, blk);
  return (int)hipGetLastError();
}

// One instantiation per n of evaluator family F (Endgame or DenseEndgame).
template <template <int> class F>
int endgame_dispatch(int n, const KArgs &a, const int2 *blk, int blocks, hipStream_t s) {
  switch (n) {
    case 1: return endgame_launch<1, F<1>>(a, blk, blocks, s);
    case 2: return endgame_launch<2, F<2>>(a, blk, blocks, s);
    case 3: return endgame_launch<3, F<3>>(a, blk, blocks, s);
    case 4: return endgame_launch<4, F<4>>(a, blk, blocks, s);
    case 5: return endgame_launch<5, F<5>>(a, blk, blocks, s);
    case 6: return endgame_launch<6, F<6>>(a, blk, blocks, s);
    case 7: return endgame_launch<7, F<7>>(a, blk, blocks, s);
    case 8: return endgame_launch<8, F<8>>(a, blk, blocks, s);
    case 9: return endgame_launch<9, F<9>>(a, blk, blocks, s);
    case 10: return endgame_launch<10, F<10>>(a, blk, blocks, s);
    case 11: return endgame_launch<11, F<11>>(a, blk, blocks, s);
    case 12: return endgame_launch<12, F<12>>(a, blk, blocks, s);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

// The dense form's instantiations, in translation units of their own so
// that they compile side by side with the term form: n <= 10
// (endgame_dense.hip, which hands n = 11, 12 on) and n = 11, 12
// (endgame_dense_wide.hip).
int launch_endgame_dense(int n, const KArgs &a, const int2 *blk, int blocks, hipStream_t s);
int launch_endgame_dense_wide(int n, const KArgs &a, const int2 *blk, int blocks, hipStream_t s);

}  // namespace hp
