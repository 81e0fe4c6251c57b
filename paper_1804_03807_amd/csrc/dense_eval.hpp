// Evaluation of one equation of total degree D <= 3 from its dense
// coefficient table (every monomial of the degree, zero where absent; the
// layout is described in hp_internal.hpp): the value in nested (Horner) form
//   f = c + sum_a x_a T_a,   T_a = l_a + sum_{b>=a} x_b S_ab,
//   S_ab = q_ab + sum_{c>=b} k_abc x_c,
// and the gradient in reverse mode over the same form: df/dx_a += T_a,
// df/dx_b += x_a S_ab, df/dx_c += x_a x_b k_abc (repeated indices give the
// multiplicities of squares and cubes by themselves).  Two complex
// multiply-adds per cubic monomial, every variable index a compile-time
// constant, so the point and the gradient are register arrays.  Used by the
// dense trackers (dense_track.hpp) and by the end game of their paths
// (endgame.hip).
#pragma once

#include "lane_track.hpp"  // cptr, sfor

namespace hp {

// Table positions of an equation in N unknowns (the host fills the table in
// the same order): constant, x_a, x_a x_b (a <= b), x_a x_b x_c
// (a <= b <= c).
template <int N>
struct DenseTable {
  static constexpr int kQuad = 1 + N;                     // first x_a x_b
  static constexpr int kCubic = kQuad + N * (N + 1) / 2;  // first x_a x_b x_c
  __device__ static constexpr int quad_at(int va, int vb) {
    return kQuad + va * N - va * (va - 1) / 2 + (vb - va);
  }
  __device__ static constexpr int cubic_at(int va, int vb, int vc) {
    int k = kCubic;
    for (int u = 0; u < va; ++u) k += (N - u) * (N - u + 1) / 2;
    for (int u = va; u < vb; ++u) k += N - u;
    return k + (vc - vb);
  }
  __device__ __forceinline__ static cd coef(cptr<double> c, int k) { return {c[2 * k], c[2 * k + 1]}; }
};

// Value of the equation whose table starts at c, at x; its gradient into g.
template <int N, int D>
__device__ __forceinline__ cd dense_equation(cptr<double> c, const cd (&x)[N], cd (&g)[N]) {
  using T = DenseTable<N>;
#pragma unroll
  for (int v = 0; v < N; ++v) g[v] = {0.0, 0.0};
  cd f = T::coef(c, 0);
  sfor<0, N>([&](auto ia) {
    constexpr int va = decltype(ia)::value;
    // T_a, complete once its b loop is done: folded into f and df/dx_a
    cd Ta = T::coef(c, 1 + va);
    if constexpr (D >= 2) {
      sfor<va, N>([&](auto ib) {
        constexpr int vb = decltype(ib)::value;
        cd S = T::coef(c, T::quad_at(va, vb));
        if constexpr (D >= 3) {
          // two partial sums shorten the dependent chain
          const cd P = cmul(x[va], x[vb]);
          cd S1 = {0.0, 0.0};
          sfor<vb, N>([&](auto ic) {
            constexpr int vc = decltype(ic)::value;
            const cd k = T::coef(c, T::cubic_at(va, vb, vc));
            if constexpr (((vc - vb) & 1) != 0) S1 = cfma(S1, k, x[vc]);
            else S = cfma(S, k, x[vc]);
            g[vc] = cfma(g[vc], P, k);
          });
          S = cadd(S, S1);
        }
        Ta = cfma(Ta, x[vb], S);
        g[vb] = cfma(g[vb], x[va], S);
      });
    }
    f = cfma(f, x[va], Ta);
    g[va] = cadd(g[va], Ta);
  });
  return f;
}

}  // namespace hp
