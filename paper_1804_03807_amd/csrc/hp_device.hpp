// Complex FP64 helpers shared by the tracker kernels (device code only).
#pragma once

#include <stdint.h>

#ifndef __HIPCC_RTC__  // hiprtc declares the HIP device API itself
#include <hip/hip_runtime.h>
#endif

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
// acc + a*b
__device__ __forceinline__ cd cfma(cd acc, cd a, cd b) {
  return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
// acc + a*r, r real
__device__ __forceinline__ cd cfma_r(cd acc, cd a, double r) {
  return {fma(a.re, r, acc.re), fma(a.im, r, acc.im)};
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
// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (each doubles the number of correct bits): x <- x + x (1 - d x).
__device__ __forceinline__ double rcp_nr(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}
// 1/b by Smith's method with Newton-refined reciprocals in place of the
// two divisions (a zero or NaN b gives a non-finite result, as 1/0 would).
__device__ __forceinline__ cd crecip_nr(cd b) {
  const bool big_re = fabs(b.re) >= fabs(b.im);
  const double p = big_re ? b.re : b.im;  // larger component
  const double q = big_re ? b.im : b.re;
  const double r = q * rcp_nr(p);
  const double id = rcp_nr(fma(q, r, p));
  return big_re ? cd{id, -r * id} : cd{r * id, -id};
}
// c ? a : b, component-wise (a conditional on the struct itself would go
// through stack temporaries)
__device__ __forceinline__ cd csel(bool c, cd a, cd b) { return {c ? a.re : b.re, c ? a.im : b.im}; }
__device__ __forceinline__ double cabs1(cd a) { return fabs(a.re) + fabs(a.im); }
__device__ __forceinline__ double cmod(cd a) { return sqrt(a.re * a.re + a.im * a.im); }
// max that propagates NaN from a (NaN never compares <=)
__device__ __forceinline__ double nmax(double m, double a) { return (a <= m) ? m : a; }

__device__ __forceinline__ cd ld(const double2 *p) {
  double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, cd v) { *p = make_double2(v.re, v.im); }
__device__ __forceinline__ void lds_add(double2 *p, cd v) {
  double *q = (double *)p;
  __hip_atomic_fetch_add(q, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(q + 1, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_add2(double *re, double *im, cd v) {
  __hip_atomic_fetch_add(re, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(im, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
// Orders the LDS accesses of the (single-wavefront) workgroup.
__device__ __forceinline__ void wsync() { __syncthreads(); }


// LDS-address-space views.  Pointers held in these types stay LDS pointers
// through selects and phis, so their accesses are ds_* instructions (a
// generic pointer the compiler cannot prove to be LDS becomes a flat access,
// which waits on both the memory and the LDS counters).
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) d2v lds_d2v;
typedef __attribute__((address_space(3))) double lds_double;
__device__ __forceinline__ cd ldl(const lds_char *p) {
  const d2v v = *(const lds_d2v *)p;
  return {v.x, v.y};
}
__device__ __forceinline__ void stl(lds_char *p, cd c) {
  d2v v = {c.re, c.im};
  *(lds_d2v *)p = v;
}
__device__ __forceinline__ void addl(lds_char *p, cd c) {
  lds_double *q = (lds_double *)p;
  __hip_atomic_fetch_add(q, c.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(q + 1, c.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Compile-time loop: f(Int<I>{}) for I = B .. E-1.  Unlike an unrolled
// runtime loop this cannot be left rolled, so register arrays indexed by I
// stay in registers (a loop whose bounds depend on an outer loop's index is
// not always fully unrolled, and its array accesses then go to scratch).
template <int V>
struct Int {
  static constexpr int value = V;
};
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(Int<B>{});
    sfor<B + 1, E>(f);
  }
}

// Right-hand side an evaluation assembles: -H_t (RK4 stages), H (Newton
// corrector) or f (end game at t = 1).
enum EvalMode { EV_NEG_HT = 0, EV_H = 1, EV_F = 2 };

}  // namespace hp
