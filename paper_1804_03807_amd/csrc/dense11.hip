// Dense tracker kernel for systems of exactly n = 11 (dense_track.hpp); a
// translation unit of its own so that it compiles beside the others.
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

namespace hp {

__global__ void __launch_bounds__(64) k_dense11(KArgs a) {
  __shared__ __align__(16) char rk[RkLds<11>::kBytes];
  const int first_sys = blockIdx.x % a.n_systems;
  for (int v = 0; v < a.n_systems; ++v) dense_drain<11>(a, (first_sys + v) % a.n_systems, (lds_char *)rk);
}

}  // namespace hp

int hp_launch_dense11(const hp::KArgs &a, int groups, void *stream) {
  hipLaunchKernelGGL(hp::k_dense11, dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int hp_dense11_per_cu(int *out) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, hp::k_dense11, 64, 0);
}
