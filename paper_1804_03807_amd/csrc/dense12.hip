// Dense tracker kernel for systems of exactly n = 12 (dense_track.hpp); a
// translation unit of its own so that it compiles beside the others.
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

namespace hp {

__global__ void __launch_bounds__(64) k_dense12(KArgs a) {
  __shared__ __align__(16) char rk[RkLds<12>::kBytes];
  const int first_sys = blockIdx.x % a.n_systems;
  for (int v = 0; v < a.n_systems; ++v) dense_drain<12>(a, (first_sys + v) % a.n_systems, (lds_char *)rk);
}

}  // namespace hp

int hp_launch_dense12(const hp::KArgs &a, int groups, void *stream) {
  hipLaunchKernelGGL(hp::k_dense12, dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int hp_dense12_per_cu(int *out) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, hp::k_dense12, 64, 0);
}
