// Serving form of the dense tracker kernels for n = 11 and 12 (see
// dense_sliced.hip).
#include <hip/hip_runtime.h>

#include "dense_track.hpp"

int hp_launch_dense_wide_sliced(int n, const hp::KArgs &a, int groups, void *stream) {
  return n == 11 ? hp::dense_launch(hp::k_dense_n<11, true>, a, groups, stream)
                 : hp::dense_launch(hp::k_dense_n<12, true>, a, groups, stream);
}

int hp_dense_wide_sliced_per_cu(int n, int *out) {
  return n == 11 ? hp::dense_per_cu(hp::k_dense_n<11, true>, out)
                 : hp::dense_per_cu(hp::k_dense_n<12, true>, out);
}
