// Complex double-double arithmetic for the device: a value is hi + lo with
// |lo| <= ulp(hi) / 2 (Dekker; Knuth, TAOCP vol. 2, 4.2.2), about 32 decimal
// digits.  Used by the end game (endgame.hip) and the double-double tracker
// (ddtrack.hip).
//
// The error-free transformations are exact only if every sum and product is
// rounded on its own: no multiply-add may be contracted into a fused one
// behind the code's back (hipcc contracts across statements by default), so
// contraction is switched off for the rest of every file that includes this
// header.  The fused products that are meant are written as fma().
#pragma once

#pragma clang fp contract(off)

#include "hp_device.hpp"

namespace hp {

struct dd {
  double hi, lo;
};
struct cdd {
  dd re, im;
};

// s + e = a + b exactly (Knuth's branch-free two-sum)
__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double v = s - a;
  return {s, (a - (s - v)) + (b - v)};
}
// s + e = a + b exactly, for |a| >= |b| (Dekker)
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd to_dd(double a) { return {a, 0.0}; }
// sum of two double-double values, both parts added error-free
__device__ __forceinline__ dd ddadd(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s = quick_two_sum(s.hi, s.lo + t.hi);
  return quick_two_sum(s.hi, s.lo + t.lo);
}
__device__ __forceinline__ dd ddneg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd ddsub(dd a, dd b) { return ddadd(a, ddneg(b)); }
// product; the exact product of the high parts from one fused multiply-add,
// the cross terms in double, lo * lo dropped
__device__ __forceinline__ dd ddmul(dd a, dd b) {
  const double p = a.hi * b.hi;
  const double e = fma(a.hi, b.hi, -p);
  return quick_two_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}
// product with a double
__device__ __forceinline__ dd ddmul_d(dd a, double b) {
  const double p = a.hi * b;
  const double e = fma(a.hi, b, -p);
  return quick_two_sum(p, e + a.lo * b);
}
// quotient: three quotient digits, each from the remainder
__device__ __forceinline__ dd dddiv(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = ddsub(a, ddmul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = ddsub(r, ddmul_d(b, q2));
  const double q3 = r.hi / b.hi;
  return ddadd(quick_two_sum(q1, q2), to_dd(q3));
}
__device__ __forceinline__ double dd_round(dd a) { return a.hi + a.lo; }

__device__ __forceinline__ cdd cddadd(cdd a, cdd b) { return {ddadd(a.re, b.re), ddadd(a.im, b.im)}; }
__device__ __forceinline__ cdd cddsub(cdd a, cdd b) { return {ddsub(a.re, b.re), ddsub(a.im, b.im)}; }
__device__ __forceinline__ cdd cddmul(cdd a, cdd b) {
  return {ddadd(ddmul(a.re, b.re), ddneg(ddmul(a.im, b.im))),
          ddadd(ddmul(a.re, b.im), ddmul(a.im, b.re))};
}
__device__ __forceinline__ cdd cddscale(cdd a, double s) { return {ddmul_d(a.re, s), ddmul_d(a.im, s)}; }
// Smith's division
__device__ __forceinline__ cdd cdddiv(cdd a, cdd b) {
  if (fabs(dd_round(b.re)) >= fabs(dd_round(b.im))) {
    const dd r = dddiv(b.im, b.re);
    const dd den = ddadd(b.re, ddmul(b.im, r));
    return {dddiv(ddadd(a.re, ddmul(a.im, r)), den), dddiv(ddsub(a.im, ddmul(a.re, r)), den)};
  }
  const dd r = dddiv(b.re, b.im);
  const dd den = ddadd(ddmul(b.re, r), b.im);
  return {dddiv(ddadd(ddmul(a.re, r), a.im), den), dddiv(ddsub(ddmul(a.im, r), a.re), den)};
}
__device__ __forceinline__ cdd to_cdd(cd z) { return {{z.re, 0.0}, {z.im, 0.0}}; }
// the nearest complex double
__device__ __forceinline__ cd round_cd(cdd z) { return {z.re.hi + z.re.lo, z.im.hi + z.im.lo}; }
__device__ __forceinline__ cdd cdd_zero() { return {{0.0, 0.0}, {0.0, 0.0}}; }

}  // namespace hp
