// Duplicate-endpoint scan on the device, the post-pass of a solve: pairs
// (a, b), a < b, of CONVERGED endpoints with
//     ||x_a - x_b||_inf <= rel max(1, ||x_a||_inf),
// which mark paths that jumped onto another path's root (the paper tracks
// every path independently, Section 1, so two paths ending at one root is a
// tracking failure to be repaired by tracking both again).
//
// Three steps on the stream, with one count read back between the first two:
//   k_dup_project  every converged path's key: a real projection
//                  sum_j u_j Re x_j + v_j Im x_j with sum |u_j| + |v_j| = 1, so
//                  that |key(a) - key(b)| <= ||x_a - x_b||_inf; appended with
//                  one atomic per wavefront (ballot, popcount, mbcnt)
//   radix sort     keys with their path ids (rocPRIM through hipCUB)
//   k_dup_scan     one lane per sorted key compares its endpoint with the
//                  following ones while their keys lie within the window
//                  2 rel max(1, ||x||_inf), and appends the pairs it finds
// Endpoints are read where the tracker wrote them (no copy); the scan reads
// a window of a few neighbours per converged path, so the cost is a sort of
// the converged keys.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {
namespace {

__device__ __forceinline__ double row_norm(const double2 *x, int n) {
  double m = 0.0;
  for (int j = 0; j < n; ++j) m = nmax(m, sqrt(x[j].x * x[j].x + x[j].y * x[j].y));
  return m;
}

__global__ void __launch_bounds__(256) k_dup_project(DupArgs a) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool conv = p < a.n_paths && a.status[p] == HP_CONVERGED;
  double key = 0.0;
  if (conv) {
    const double2 *x = a.endpoints + p * a.n;
    for (int j = 0; j < a.n; ++j) key += a.w[2 * j] * x[j].x + a.w[2 * j + 1] * x[j].y;
  }
  const uint64_t m = __ballot(conv);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int first = __builtin_ctzll(m);
  unsigned long long base = 0;
  if (lane == first) base = atomicAdd(a.count, (unsigned long long)__popcll(m));
  base = __shfl(base, first);
  if (!conv) return;
  const unsigned rank =
      __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  const unsigned long long slot = base + rank;
  if (slot < (unsigned long long)a.cap) {
    a.keys[slot] = key;
    a.ids[slot] = p;
  }
}

__global__ void __launch_bounds__(256) k_dup_scan(DupArgs a, long long m) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double ki = a.keys_sorted[i];
  const long long pi = a.ids_sorted[i];
  const double2 *xi = a.endpoints + pi * a.n;
  const double ni = row_norm(xi, a.n);
  const double win = 2.0 * a.rel * (ni > 1.0 ? ni : 1.0);
  for (long long k = i + 1; k < m; ++k) {
    if (a.keys_sorted[k] - ki > win) break;
    const long long pk = a.ids_sorted[k];
    const double2 *xk = a.endpoints + pk * a.n;
    const long long pa = pi < pk ? pi : pk, pb = pi < pk ? pk : pi;
    const double na = pa == pi ? ni : row_norm(xk, a.n);
    double d = 0.0;
    for (int j = 0; j < a.n; ++j) {
      const double dr = xi[j].x - xk[j].x, di = xi[j].y - xk[j].y;
      d = nmax(d, sqrt(dr * dr + di * di));
    }
    if (d <= a.rel * (na > 1.0 ? na : 1.0)) {
      const unsigned long long slot = atomicAdd(a.pair_count, 1ull);
      if (slot < (unsigned long long)a.max_pairs) {
        a.pairs[2 * slot] = pa;
        a.pairs[2 * slot + 1] = pb;
      }
    }
  }
}

// Paths tracked again: result k goes to path ids[k] of the full outputs.
__global__ void __launch_bounds__(256) k_scatter(const long long *ids, long long m, int n,
                                                 const double2 *e_src, const int32_t *s_src,
                                                 const hp_path_stats *st_src, double2 *e_dst,
                                                 int32_t *s_dst, hp_path_stats *st_dst) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const long long p = ids[k];
  for (int j = 0; j < n; ++j) e_dst[p * n + j] = e_src[k * n + j];
  s_dst[p] = s_src[k];
  if (st_dst) st_dst[p] = st_src[k];
}

unsigned grid_of(long long items, int block) {
  return (unsigned)((items + block - 1) / block);
}

}  // namespace
}  // namespace hp

using hp::DupArgs;

size_t hp_dup_sort_temp_bytes(long long cap) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const double *)nullptr, (double *)nullptr,
                                           (const long long *)nullptr, (long long *)nullptr, cap);
  return bytes;
}

int hp_launch_dup_project(const DupArgs &a, void *stream) {
  if (a.n_paths <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(hp::k_dup_project, dim3(hp::grid_of(a.n_paths, 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int hp_launch_dup_sort(const DupArgs &a, long long m, void *stream) {
  if (m <= 0) return (int)hipSuccess;
  size_t bytes = a.temp_bytes;
  return (int)hipcub::DeviceRadixSort::SortPairs(a.temp, bytes, a.keys, a.keys_sorted, a.ids,
                                                 a.ids_sorted, m, 0, 64, (hipStream_t)stream);
}

int hp_launch_dup_scan(const DupArgs &a, long long m, void *stream) {
  if (m <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(hp::k_dup_scan, dim3(hp::grid_of(m, 256)), dim3(256), 0, (hipStream_t)stream,
                     a, m);
  return (int)hipGetLastError();
}

int hp_launch_scatter(const long long *ids, long long m, int n, const double2 *e_src,
                      const int32_t *s_src, const hp_path_stats *st_src, double2 *e_dst,
                      int32_t *s_dst, hp_path_stats *st_dst, void *stream) {
  if (m <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(hp::k_scatter, dim3(hp::grid_of(m, 256)), dim3(256), 0, (hipStream_t)stream,
                     ids, m, n, e_src, s_src, st_src, e_dst, s_dst, st_dst);
  return (int)hipGetLastError();
}
