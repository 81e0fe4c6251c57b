// Solve of a small complex system held entirely in registers, for the
// one-path-per-lane kernels whose Jacobian is a register array (the
// specialised and the dense kernels).
#pragma once

#include "hp_device.hpp"

namespace hp {

// true, through an empty asm on a scalar register: a wave-uniform branch
// condition the compiler can neither fold nor merge with another
__device__ __forceinline__ bool opaque_true() {
  int v = 1;
  asm volatile("" : "+s"(v));
  return v != 0;
}

// LU with partial pivoting (largest |re|+|im| in the column, ties to the
// lowest row) on the registers, then back substitution into dx.  A row
// exchange is a select per entry: the pivot row is data dependent and
// registers cannot be indexed by a lane-varying value.  sing: an exactly
// zero (or NaN) pivot.  Lanes with live false discard dx and sing (lanes
// whose paths have ended, or whose corrector has stopped, still run the
// solve in step with the others).  With SkipRows the exchange of a row is
// skipped for the whole wavefront when no live lane takes its pivot there.
// In the dense kernels the branches this adds also cut the register spills;
// in the specialised kernel of n = 10, which spills already, they cost more
// than they save (and n = 9, which spills too, keeps the exchanges as well).
//
// With RowBlocks the elimination of each row sits behind a wave-uniform
// branch whose condition the compiler cannot evaluate (always true): every
// row becomes a block of its own, which keeps the scheduler from
// interleaving rows and lowers the register pressure in the dense kernel
// for n <= 10 (fewer spills, 13 % less time on a batch of dense systems);
// the specialised kernels run slower with it (n = 8) or spill more
// (n = 9, 10), and so do the dense kernels of n = 11, 12 on the serving
// sample, where they carry most of the paths.
template <int N, bool SkipRows, bool RowBlocks>
__device__ __forceinline__ void reg_lu_solve(cd (&J)[N][N], cd (&b)[N], cd dx[N], bool &sing,
                                             bool live) {
  // compile-time loops throughout: with bounds that depend on the column k,
  // unrolled runtime loops are not always unrolled fully, and J would then
  // be indexed at run time and live in scratch memory
  sing = false;
  sfor<0, N>([&](auto ik) {
    constexpr int k = decltype(ik)::value;
    double best = -1.0;
    int p = k;
    sfor<k, N>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const double c = cabs1(J[i][k]);
      const bool take = c > best;
      best = take ? c : best;
      p = take ? i : p;
    });
    if (!(best > 0.0)) sing = true;
    sfor<k + 1, N>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const bool sw = (i == p);
      if (SkipRows && ballot(live && sw) == 0) return;
      sfor<k, N>([&](auto ij) {
        constexpr int j = decltype(ij)::value;
        const cd u = J[k][j], v = J[i][j];
        J[k][j] = csel(sw, v, u);
        J[i][j] = csel(sw, u, v);
      });
      const cd u = b[k], v = b[i];
      b[k] = csel(sw, v, u);
      b[i] = csel(sw, u, v);
    });
    const cd inv = crecip_nr(J[k][k]);
    J[k][k] = inv;  // kept for the back substitution
    sfor<k + 1, N>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      if (RowBlocks && !opaque_true()) return;
      const cd l = cmul(J[i][k], inv);
      sfor<k + 1, N>([&](auto ij) {
        constexpr int j = decltype(ij)::value;
        J[i][j] = cfms(J[i][j], l, J[k][j]);
      });
      b[i] = cfms(b[i], l, b[k]);
    });
  });
  sfor<0, N>([&](auto ir) {
    constexpr int k = N - 1 - decltype(ir)::value;
    cd y = b[k];
    sfor<k + 1, N>([&](auto ij) {
      constexpr int j = decltype(ij)::value;
      y = cfms(y, J[k][j], dx[j]);
    });
    dx[k] = cmul(y, J[k][k]);
  });
}

}  // namespace hp
