// Internal layouts shared by the device kernels and the host side of
// libhomotopy.  Nothing here is part of the C ABI.
#pragma once

#include <stdint.h>

#ifndef __HIPCC_RTC__  // hiprtc declares the HIP device API itself
#include <hip/hip_runtime.h>

#include <string>
#endif

#include "homotopy.h"

namespace hp {

constexpr int kLanes = 64;  // CDNA wavefront width: one path per lane
// The terms of a system are sorted by their number of factors k; the kp
// array holds kKSlots entries per system: the system's terms with k factors
// are its terms kp[k] .. kp[k+1]-1, counted from its first term.
constexpr int kKSlots = HP_MAX_N + 2;

// One term c * prod x_v^e of equation i.  On the device the coefficient and
// the 16-byte factor word live in two arrays (16-byte strides keep the lanes
// of a group on distinct LDS banks).  Factor word: byte 0 = number of
// factors k (<= HP_MAX_N) in its low bits, plus kChunkUniform when every
// term of the term's chunk (the n consecutive terms of its k class that one
// group of n lanes takes at once) belongs to the same equation; bytes 1..k =
// (v | e << 4), byte 15 = equation i.
constexpr uint32_t kChunkUniform = 0x80;
struct alignas(32) DevTerm {
  double cre, cim;
  uint32_t w[4];
};

// Per-system descriptor, read with scalar loads by a workgroup that works on
// the system.
struct alignas(16) DevSys {
  int32_t n;          // unknowns
  int32_t emax;       // largest exponent of any variable in any term
  int32_t eq_base;    // index of this system's kKSlots block in the kp array
  int32_t root_base;  // index of the first root of unity of this system
  int32_t term_base;  // index of the first term of this system
  int32_t n_terms;    // terms of this system (staged in LDS if <= kMaxStagedTerms)
  int32_t deg[HP_MAX_N];       // equation degrees d_i
  int32_t root_off[HP_MAX_N];  // roots of x_i^{d_i} = 1 start at root_base + root_off[i]
  int64_t radix[HP_MAX_N];     // prod_{j<i} d_j
  double gre, gim;             // gamma
  int64_t n_paths;             // queue length of this system
  int64_t out_path_base;       // first status/stats index of this system
  int64_t out_x_base;          // first endpoint (hp_c64) index of this system
  const int64_t *ids;          // queue index -> path id (nullptr: id_base + index)
  int64_t id_base;
  const int64_t *slots;        // queue index -> output slot (nullptr: the index);
                               // a slot holds a suspended path's state (serving)
  // general start system g (g_n_terms == 0: total degree, g_i = x_i^{d_i} - 1)
  int32_t g_term_base;         // first term of g
  int32_t g_n_terms;
  int32_t g_eq_base;           // g's kKSlots block in the kp array
  int32_t g_pad;
  const double2 *start;        // [path id][n] start points (nullptr: roots of unity)
  // dense table (systems of total degree <= 3 on the dense kernel): the
  // coefficients of equation i start at dense_base + dense_off[i], see
  // kDenseMaxN
  int32_t dense_base;
  int32_t dense_off[HP_MAX_N];
  int32_t dense_pad[3];
  // end game at t = 1: f's terms once more, in equation order, in the same
  // term arrays: equation i owns terms eg_base + eg_ptr[i] ..
  // eg_base + eg_ptr[i+1] - 1
  int32_t eg_base;
  int32_t eg_ptr[HP_MAX_N + 1];
  int32_t eg_pad[2];
  // the end game's compacted list of this system's paths to refine starts
  // at this entry (64 entries per block of its queue)
  int64_t eg_list_base;
  int64_t eg_list_pad;
};

// Dense kernel: systems of n <= kDenseMaxN unknowns whose equations have
// total degree <= 3, every equation's coefficients as a full table in the
// fixed order constant; x_a (a < n); x_a x_b (a <= b); x_a x_b x_c
// (a <= b <= c), each block present up to the equation's degree, loops with
// a outermost (missing monomials hold zero).
constexpr int kDenseMaxN = 10;      // k_dense: any n up to this in one launch
constexpr int kDenseWideMaxN = 12;  // k_dense_n<11>, k_dense_n<12>: one exact n per launch
constexpr int kDenseMaxDeg = 3;

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
  const double2 *tcoef;  // term coefficients
  const uint4 *tmeta;    // term factor words
  const int32_t *eqp;    // kp blocks: kKSlots term offsets per system
  const double2 *roots;  // roots of unity, (cos, sin)
  unsigned long long *qhead;  // per system queue heads (persistent mode)
  double2 *endpoints;
  int32_t *status;
  hp_path_stats *stats;  // may be null
  DevTol tol;
  int32_t stage;         // group kernels: copy term tables of <= kMaxStagedTerms into LDS
  PlainState ps;         // plain mode only
  const double2 *dcoef;  // dense coefficient tables (dense kernel)
  double2 *endpoints_lo; // low parts of the endpoints (double-double tracker)
  int32_t step_budget;   // serving kernels: steps per wavefront in this launch (0: until
                         // the queues are drained); past it, paths in flight are
                         // suspended to their slots
  int32_t lane_paths;    // specialised and dense kernels: lanes 0 .. lane_paths - 1 of a
                         // wavefront hold paths (0: all 64), a tuning choice
  const double2 *pcoef;  // specialised kernels in the coefficient-parameter form:
                         // (cf, cg, gamma cg - cf) per term, in packed term order
  const long long *eg_list;  // end game over a list: per system, from its eg_list_base, the
  const unsigned *eg_count;  // queue indices of the paths to refine (k_eg_select); per
                             // system their number
};

// Lanes of a wavefront that take paths from the refill queue in the
// one-path-per-lane kernels whose paths per wavefront are a launch argument.
__device__ __forceinline__ bool lane_holds_path(const KArgs &a) {
  return (int)(threadIdx.x & 63) < (a.lane_paths > 0 ? a.lane_paths : kLanes);
}

// Status codes of a slot that holds a suspended path (serving) or a path not
// started yet; a finished path's status is its hp_status (>= 0).
constexpr int32_t kSuspendedTrack = -2;
constexpr int32_t kSuspendedFinal = -3;
constexpr int32_t kUnstarted = -4;

enum Mode : int32_t { M_IDLE = 0, M_TRACK = 1, M_FINAL = 2 };

// Arguments of the duplicate-endpoint scan (dedup.hip).
struct DupArgs {
  int32_t n;
  long long n_paths;
  const double2 *endpoints;  // [n_paths][n]
  const int32_t *status;     // [n_paths]
  double rel;
  double w[2 * HP_MAX_N];    // projection weights (re, im) per unknown, sum |w| = 1
  double *keys;              // [cap] projections of the converged paths
  long long *ids;            // [cap] their path indices
  double *keys_sorted;       // [cap]
  long long *ids_sorted;     // [cap]
  long long cap;
  unsigned long long *count;       // converged paths seen (may exceed cap)
  long long *pairs;                // [2 max_pairs]
  long long max_pairs;
  unsigned long long *pair_count;  // pairs found (may exceed max_pairs)
  void *temp;                      // radix sort workspace
  size_t temp_bytes;
};

// Arguments of the serving harvest (serve.hip): entry k of the launch's
// queues owns arena path slot path_slot[k] (status, stats) and endpoint
// coordinates x_off[k] .. x_off[k] + n[k] - 1; finished entries become
// records 0 .. *count - 1.
struct CollectArgs {
  long long m;
  const long long *path_slot;
  const long long *x_off;
  const int32_t *n;
  int32_t *status;           // arena
  const double2 *endpoints;  // arena
  const hp_path_stats *stats;
  int32_t *rec_entry;        // [m]
  int32_t *rec_status;       // [m]
  double2 *rec_x;            // [m][HP_MAX_N]
  hp_path_stats *rec_stats;  // [m]
  unsigned *count;
};

// Kernel variants compiled into the library: the register arrays hold up to
// n_max unknowns; a system of n unknowns runs on the smallest n_max >= n.
constexpr int kNmaxVariants[] = {4, 8, 10, 12};

// LDS layout of a workgroup (one wavefront): a 64-entry refill broadcast,
// then one region per lane group (floor(64/n) groups plus one spare group
// for the lanes past the last full group).
constexpr size_t kCtlBytes = 64 * 8;
// Fixed part of a group's region, laid out for the n_max of the kernel so
// that every access is a compile-time offset from one base address; the
// power table [n][emax] follows it.
template <int NMAX>
struct GroupLds {
  double Jre[NMAX][NMAX + 1];  // Jacobian accumulator, real parts (rows padded)
  double Jim[NMAX][NMAX + 1];  // imaginary parts
  double fre[NMAX], fim[NMAX];  // f values
  double gre[NMAX], gim[NMAX];  // g values (general start system)
  double2 prow[NMAX + 1]; // normalised pivot row, [NMAX] = right-hand side
  double2 dsol[NMAX];     // solution of the last linear solve
  double cand[NMAX];      // pivot candidates
  double red[2 * NMAX];   // reductions
};
__host__ __device__ constexpr size_t group_fixed_bytes(int nmax) {
  return (size_t)16 * ((size_t)nmax * (nmax + 1) + 4 * nmax + 1) + (size_t)8 * 3 * nmax;
}
// Stride of one group's region: the fixed part and the power table, padded
// to an odd number of 16-byte units, so that up to 16 groups of a wavefront
// start on distinct 16-byte bank quads (a multiple of 256 bytes would put
// every group's copy of an entry on the same banks).
__host__ __device__ constexpr size_t group_lds_bytes(int nmax, int emax) {
  return (((group_fixed_bytes(nmax) + (size_t)16 * nmax * emax + 15) / 16) | 1) * 16;
}
static_assert(sizeof(GroupLds<8>) == group_fixed_bytes(8), "layout");
static_assert(sizeof(GroupLds<10>) == group_fixed_bytes(10), "layout");
static_assert(sizeof(GroupLds<12>) == group_fixed_bytes(12), "layout");
// Term tables up to this size are staged in LDS at kernel start.
constexpr int kMaxStagedTerms = 512;
// LDS bytes of a workgroup running a system of n unknowns and n_terms
// terms on the n_max variant: staged terms (if they fit), then floor(64/n)
// groups plus one spare group.
inline size_t staged_term_bytes(int n_terms) {
  return n_terms <= kMaxStagedTerms ? (size_t)n_terms * 32 : 0;
}
inline size_t system_lds_bytes(int nmax, int n, int emax, int n_terms, bool stage) {
  return kCtlBytes + (stage ? staged_term_bytes(n_terms) : 0) +
         (size_t)(kLanes / n + 1) * group_lds_bytes(nmax, emax);
}

// Lane-per-path kernels (lanes.hip): every lane tracks its own path; one
// instantiation per exact n (1..8) with PW = 64 paths per wavefront, and
// PW = 32 for n = 7, 8 (systems whose power table is large).  LDS per
// wavefront: [J | rhs] and the power table, each entry PW * 16 bytes.
struct LaneVariant {
  int n, pw;
};
constexpr LaneVariant kLaneVariants[] = {{1, 64}, {2, 64}, {3, 64}, {4, 64}, {5, 64},
                                         {6, 64}, {7, 64}, {8, 64}, {7, 32}, {8, 32}};
inline size_t lanes_lds_bytes(int n, int pw, int emax) {
  return (size_t)(n * (n + 1) + n * emax) * (size_t)pw * 16;
}

}  // namespace hp

// Kernel launchers (tracker.hip, lanes.hip, dense.hip, dense11.hip, dense12.hip,
// dense_sliced.hip, dense_wide_sliced.hip, endgame.hip, dedup.hip, dedup_static.hip, ddtrack.hip, serve.hip).  Return a hipError_t
// value.
extern "C++" {
// general: the systems use a general start system or explicit start points
int hp_launch_persistent(int nmax, bool general, const hp::KArgs &a, int groups, size_t lds,
                         void *stream);
int hp_launch_plain_init(const hp::KArgs &a, void *stream);
int hp_launch_plain_step(int nmax, bool general, const hp::KArgs &a, int groups, size_t lds,
                         void *stream);
int hp_max_groups_per_cu(int nmax, bool general, size_t lds, int *out);
int hp_launch_lanes(int n, int pw, const hp::KArgs &a, int groups, size_t lds, void *stream);
int hp_launch_lanes_plain(int n, int pw, const hp::KArgs &a, int groups, size_t lds,
                          void *stream);
int hp_lanes_per_cu(int n, int pw, size_t lds, int *out);
int hp_launch_dense(const hp::KArgs &a, int groups, void *stream);
int hp_dense_per_cu(int *out);
int hp_launch_dense11(const hp::KArgs &a, int groups, void *stream);
int hp_dense11_per_cu(int *out);
int hp_launch_dense12(const hp::KArgs &a, int groups, void *stream);
int hp_dense12_per_cu(int *out);
// Serving forms of the dense kernels (dense_sliced.hip, dense_wide_sliced.hip;
// n = 11 or 12 for the wide one).
int hp_launch_dense_sliced(const hp::KArgs &a, int groups, void *stream);
int hp_dense_sliced_per_cu(int *out);
int hp_launch_dense_wide_sliced(int n, const hp::KArgs &a, int groups, void *stream);
int hp_dense_wide_sliced_per_cu(int n, int *out);
// Duplicate scan (dedup.hip): projection and compaction of the converged
// endpoints, radix sort of m keys, window scan over the m sorted keys; and
// the scatter of re-tracked results into the full outputs.
size_t hp_dup_sort_temp_bytes(long long cap);
int hp_launch_dup_project(const hp::DupArgs &a, void *stream);
int hp_launch_dup_sort(const hp::DupArgs &a, long long m, void *stream);
int hp_launch_dup_scan(const hp::DupArgs &a, long long m, void *stream);
#ifndef __HIPCC_RTC__
// The duplicate scan in the library's static per-GPU workspace
// (dedup_static.hip), allocating nothing: 0, -1 (device error, text in err)
// or -2 (more converged endpoints than the workspace holds).  Pairs go to
// a.pairs (up to a.max_pairs), their number to *n_pairs.
long long hp_dup_static_max_converged();
int hp_dup_static_scan(int device, hp::DupArgs a, long long *n_pairs, std::string &err,
                       void *stream);
#endif
int hp_launch_scatter(const long long *ids, long long m, int n, const double2 *e_src,
                      const int32_t *s_src, const hp_path_stats *st_src, double2 *e_dst,
                      int32_t *s_dst, hp_path_stats *st_dst, void *stream);
// Double-double tracker (ddtrack.hip): one system of n unknowns, n lanes
// per path; resident workgroups per CU of its n instantiation.
int hp_launch_ddtrack(int n, const hp::KArgs &a, int groups, void *stream);
int hp_ddtrack_per_cu(int n, int *out);
// Serving harvest of finished paths, and a fill of m int32 values (serve.hip).
int hp_launch_collect(const hp::CollectArgs &a, void *stream);
int hp_launch_fill_i32(int32_t *p, long long m, int32_t v, void *stream);
// End game of the paths of systems with n unknowns: blk[b] = (system, first
// queue index) of block b (64 paths each), or blk == nullptr for one system
// (system 0, block b from queue index 64 b); with a.eg_list set, the block
// takes the same positions of its system's compacted list instead.  dense:
// the systems' dense tables (a.dcoef) evaluate f and J_f, else their
// equation-ordered terms.
int hp_launch_endgame(int n, const hp::KArgs &a, const int2 *blk, int blocks, bool dense,
                      void *stream);
// Compacts, per system, the queue indices of `blocks` blocks (blk as for
// hp_launch_endgame) whose paths the end game refines (CONVERGED or
// FAILED_NEWTON_T1) into list from the system's eg_list_base, their number
// into counts[system] (zeroed by the caller).
int hp_launch_eg_select(const hp::KArgs &a, const int2 *blk, int blocks, long long *list,
                        unsigned *counts, void *stream);
}
