// Harvest step of the serving loop: after a launch whose wavefronts may have
// stopped on their step budget, the paths of the launch's queues that
// finished are copied out of their slots into compact records (one atomic
// per wavefront: ballot, popcount, mbcnt), and their slots are marked free
// (kUnstarted), so that the host reads back only finished paths.  Slots of
// suspended or unstarted paths are left as they are.
#include <hip/hip_runtime.h>

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {
namespace {

__global__ void __launch_bounds__(256) k_collect(CollectArgs a) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long ps = 0;
  int st = -1;
  if (k < a.m) {
    ps = a.path_slot[k];
    st = a.status[ps];
  }
  const bool fin = st >= 0;
  const uint64_t m = __ballot(fin);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int first = __builtin_ctzll(m);
  unsigned base = 0;
  if (lane == first) base = atomicAdd(a.count, (unsigned)__popcll(m));
  base = __shfl(base, first);
  if (!fin) return;
  const unsigned r = base + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  a.rec_entry[r] = (int32_t)k;
  a.rec_status[r] = st;
  a.rec_stats[r] = a.stats[ps];
  const double2 *x = a.endpoints + a.x_off[k];
  double2 *y = a.rec_x + (long long)r * HP_MAX_N;
  const int n = a.n[k];
  for (int j = 0; j < n; ++j) y[j] = x[j];
  a.status[ps] = kUnstarted;
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *p, long long m, int32_t v) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) p[k] = v;
}

}  // namespace
}  // namespace hp

int hp_launch_collect(const hp::CollectArgs &a, void *stream) {
  if (a.m <= 0) return (int)hipSuccess;
  const unsigned blocks = (unsigned)((a.m + 255) / 256);
  hipLaunchKernelGGL(hp::k_collect, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int hp_launch_fill_i32(int32_t *p, long long m, int32_t v, void *stream) {
  if (m <= 0) return (int)hipSuccess;
  const unsigned blocks = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(hp::k_fill_i32, dim3(blocks), dim3(256), 0, (hipStream_t)stream, p, m, v);
  return (int)hipGetLastError();
}
