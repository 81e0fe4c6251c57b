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
// Terms.  Each term c x^a is differentiated in reverse mode: prefix
// products from the coefficient, then a backward sweep of suffix products
// that starts from t, so that the partial derivatives arrive already scaled
// by t while the term value stays unscaled (H_t = f - gamma g needs f
// itself).  They are added into the lane's own entries (ds_add_f64: no
// other lane touches them).  The linear systems are solved by LU with
// partial pivoting (largest |re|+|im|, ties to the lowest row) on the LDS
// rows of the lane; row exchanges only swap the row addresses each lane
// keeps in registers.  Path state, step control and scheduling are shared
// with the other lane kernels (lane_track.hpp).
#include <hip/hip_runtime.h>

#include "lane_track.hpp"

namespace hp {

// PW: lanes that hold paths (lanes PW..63 stay idle).
template <int N, int PW>
struct Lanes : LaneTrack<Lanes<N, PW>, N> {
  using Base = LaneTrack<Lanes<N, PW>, N>;
  using Base::a;
  using Base::lane;
  using Base::slot;
  using Base::sp;
  using Base::deg;
  using Base::gamma;
  using Base::xc;
  static constexpr int NMAX = N;
  static constexpr int n = N;
  static constexpr int kCols = NMAX + 1;     // J columns + right-hand side
  static constexpr int kEntry = PW * 16;     // bytes of one entry
  static constexpr int kJ = NMAX * kCols;    // entries of [J | rhs]

  lds_char *base;   // this lane's double2 in entry 0
  // ---- current system (wave-uniform) ----
  int emax;
  const double2 *tcoef;  // this system's terms (vector loads: their wait
  const uint4 *tmeta;    // counter is not shared with the LDS atomics)
  int kpv[N + 2];  // terms with k factors are this system's terms kpv[k] .. kpv[k+1]-1

  __device__ Lanes(const KArgs &args, char *smem) : Base(args, (threadIdx.x & 63) < PW) {
    base = (lds_char *)smem + (slot ? lane : 0) * 16;
  }

  // ---- LDS entries of this lane ----
  __device__ __forceinline__ lds_char *ent(int e) const { return base + e * kEntry; }
  __device__ __forceinline__ lds_char *jent(int i, int j) const { return ent(i * kCols + j); }
  __device__ __forceinline__ lds_char *xpent(int v, int e1) const { return ent(kJ + v * emax + e1); }

  __device__ __forceinline__ void load_system(int s) {
    this->load_common(s);
    emax = sp->emax;
    tcoef = a.tcoef + sp->term_base;
    tmeta = a.tmeta + sp->term_base;
    {
      cptr<int32_t> kp = as_const(a.eqp) + sp->eq_base;
#pragma unroll
      for (int k = 0; k <= N + 1; ++k) kpv[k] = kp[k < N + 1 ? k : HP_MAX_N + 1];
    }
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
  __device__ __forceinline__ void solve(cd dx[NMAX], bool &sing, bool /*live*/) {
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

  // max_i |rhs_i| (after an EV_F evaluation: the residual ||f(x)||_inf)
  __device__ __forceinline__ double residual() const {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) r = nmax(r, cmod(ldl(jent(i, NMAX))));
    return r;
  }
};

// Persistent kernel (refilled from the device queue) and plain kernel (one
// step per launch); see lane_persistent and lane_plain.
template <int N, int PW>
__global__ void __launch_bounds__(64) k_lanes(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Lanes<N, PW> tr(a, smem);
  lane_persistent(a, tr);
}

template <int N, int PW>
__global__ void __launch_bounds__(64) k_lanes_plain(KArgs a) {
  extern __shared__ __align__(16) char smem[];
  Lanes<N, PW> tr(a, smem);
  lane_plain<Lanes<N, PW>, PW>(a, tr);
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
