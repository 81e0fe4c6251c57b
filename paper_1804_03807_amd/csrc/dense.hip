// Dense tracker kernel for systems of n <= kDenseMaxN (mixed n in one
// launch), as plans and batches run it (dense_track.hpp).
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

int hp_launch_dense(const hp::KArgs &a, int groups, void *stream) {
  return hp::dense_launch(hp::k_dense<false>, a, groups, stream);
}

int hp_dense_per_cu(int *out) { return hp::dense_per_cu(hp::k_dense<false>, out); }
