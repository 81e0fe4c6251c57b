// Dense tracker kernel for systems of exactly n = 12 (dense_track.hpp); a
// translation unit of its own so that it compiles beside the others.
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

int hp_launch_dense12(const hp::KArgs &a, int groups, void *stream) {
  return hp::dense_launch(hp::k_dense_n<12, false>, a, groups, stream);
}

int hp_dense12_per_cu(int *out) { return hp::dense_per_cu(hp::k_dense_n<12, false>, out); }
