// Serving form of the dense tracker kernel for n <= kDenseMaxN: paths
// suspend after a step budget and resume in a later launch
// (dense_track.hpp, lane_drain).
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

int hp_launch_dense_sliced(const hp::KArgs &a, int groups, void *stream) {
  return hp::dense_launch(hp::k_dense<true>, a, groups, stream);
}

int hp_dense_sliced_per_cu(int *out) { return hp::dense_per_cu(hp::k_dense<true>, out); }
