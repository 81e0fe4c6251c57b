// Dense tracker kernel for systems of exactly n = 11 (dense_track.hpp); a
// translation unit of its own so that it compiles beside the others.
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

int hp_launch_dense11(const hp::KArgs &a, int groups, void *stream) {
  return hp::dense_launch(hp::k_dense_n<11, false>, a, groups, stream);
}

int hp_dense11_per_cu(int *out) { return hp::dense_per_cu(hp::k_dense_n<11, false>, out); }
