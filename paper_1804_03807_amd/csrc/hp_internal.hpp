// Internal layouts shared by the device kernels and the host side of
// libhomotopy.  Nothing here is part of the C ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "homotopy.h"

namespace hp {

constexpr int kLanes = 64;  // CDNA wavefront width: one path per lane
// Per equation, terms are sorted by their number of factors k; the term
// index array holds kKSlots entries per equation: terms with k factors are
// [kp[k], kp[k+1]).
constexpr int kKSlots = HP_MAX_N + 2;

// One term c * prod x_v^e, packed for 256-bit scalar loads:
// w byte 0 = number of factors k (<= HP_MAX_N), bytes 1..k = (v | e << 4).
struct alignas(32) DevTerm {
  double cre, cim;
  uint32_t w[4];
};

// Per-system descriptor, read with scalar loads by a workgroup that works on
// the system.
struct alignas(16) DevSys {
  int32_t n;          // unknowns
  int32_t emax;       // largest exponent of any variable in any term
  int32_t eq_base;    // index of this system's first kKSlots block in the kp array
  int32_t root_base;  // index of the first root of unity of this system
  int32_t deg[HP_MAX_N];       // equation degrees d_i
  int32_t root_off[HP_MAX_N];  // roots of x_i^{d_i} = 1 start at root_base + root_off[i]
  int64_t radix[HP_MAX_N];     // prod_{j<i} d_j
  double gre, gim;             // gamma
  int64_t n_paths;             // queue length of this system
  int64_t out_path_base;       // first status/stats index of this system
  int64_t out_x_base;          // first endpoint (hp_c64) index of this system
  const int64_t *ids;          // queue index -> path id (nullptr: identity)
};

struct DevTol {
  double tol_residual, tol_corr, tol_final, div_radius, h_init, h_min, h_max;
  int32_t max_steps, max_newton, max_newton_final, pad;
};

// Per-path state of the plain (one launch per step) tracker, structure of
// arrays over the queue index so that a wavefront's 64 paths are contiguous.
struct PlainState {
  double2 *x0;   // [n][P]: accepted point, component-major
  double *t;     // [P]
  double *h;     // [P]
  int32_t *iv;   // [8][P]: mode, accepts, steps, rejections, newton, evals, solves, spare
  int64_t P;
  unsigned int *active;  // paths still tracking after the launch
};

struct KArgs {
  const DevSys *sys;
  int32_t n_systems;
  int32_t emax_all;      // LDS power table depth of the launch
  int32_t nl;            // LDS row stride: largest n of the launch
  int32_t pad;
  const DevTerm *terms;
  const int32_t *eqp;    // kp blocks: absolute term indices, kKSlots per equation
  const double2 *roots;  // roots of unity, (cos, sin)
  unsigned long long *qhead;  // per system queue heads (persistent mode)
  double2 *endpoints;
  int32_t *status;
  hp_path_stats *stats;  // may be null
  DevTol tol;
  PlainState ps;         // plain mode only
};

enum Mode : int32_t { M_IDLE = 0, M_TRACK = 1, M_FINAL = 2 };

// Kernel variants compiled into the library: (n_max, waves per workgroup),
// i.e. one or two Jacobian rows per wave.
struct Variant {
  int nmax, waves;
};
constexpr Variant kVariants[] = {{4, 2}, {4, 4}, {8, 4}, {8, 8}, {12, 6}};

// LDS shared by the Jacobian accumulators (eval) and the pivot row,
// solution and pivot candidates (solve), for row stride nl.
__host__ __device__ constexpr size_t lds_union_bytes(int nl, int waves) {
  size_t acc = (size_t)waves * nl * 16 * kLanes;
  size_t sol = ((size_t)(2 * nl + 1) * 16 + (size_t)nl * 8) * kLanes;
  return acc > sol ? acc : sol;
}
// LDS bytes of a workgroup with `waves` waves, row stride nl (largest n of
// the launch) and power tables of depth emax.
inline size_t lds_bytes(int nl, int waves, int emax) {
  return (size_t)nl * emax * 16 * kLanes + lds_union_bytes(nl, waves) +
         (size_t)2 * waves * 8 * kLanes + 64 * 8 + 64;
}

}  // namespace hp

// Kernel launchers (tracker.hip).  Return a hipError_t value.
extern "C++" {
int hp_launch_persistent(int nmax, int waves, const hp::KArgs &a, int groups, size_t lds,
                         void *stream);
int hp_launch_plain_init(int nmax, const hp::KArgs &a, void *stream);
int hp_launch_plain_step(int nmax, int waves, const hp::KArgs &a, size_t lds, void *stream);
int hp_max_groups_per_cu(int nmax, int waves, size_t lds, int *out);
}
