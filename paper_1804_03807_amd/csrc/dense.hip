// Dense tracker kernel for systems of n <= kDenseMaxN (mixed n in one
// launch): a wavefront drains the systems' refill queues one after another
// and runs the tracker instantiated for each system's n (dense_track.hpp).
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

namespace hp {

// Persistent kernel over every system of the launch; the system's n picks
// the instantiation (wave-uniform).
__global__ void __launch_bounds__(64) k_dense(KArgs a) {
  __shared__ __align__(16) char rk[RkLds<kDenseMaxN>::kBytes];
  lds_char *lds = (lds_char *)rk;
  const int first_sys = blockIdx.x % a.n_systems;
  for (int v = 0; v < a.n_systems; ++v) {
    const int s = (first_sys + v) % a.n_systems;
    switch (as_const(a.sys)[s].n) {
      case 1: dense_drain<1>(a, s, lds); break;
      case 2: dense_drain<2>(a, s, lds); break;
      case 3: dense_drain<3>(a, s, lds); break;
      case 4: dense_drain<4>(a, s, lds); break;
      case 5: dense_drain<5>(a, s, lds); break;
      case 6: dense_drain<6>(a, s, lds); break;
      case 7: dense_drain<7>(a, s, lds); break;
      case 8: dense_drain<8>(a, s, lds); break;
      case 9: dense_drain<9>(a, s, lds); break;
      case 10: dense_drain<10>(a, s, lds); break;
      default: break;  // the host admits n <= kDenseMaxN only
    }
  }
}

}  // namespace hp

using namespace hp;

int hp_launch_dense(const KArgs &a, int groups, void *stream) {
  hipLaunchKernelGGL(k_dense, dim3(groups), dim3(64), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int hp_dense_per_cu(int *out) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_dense, 64, 0);
}
