// End game kernels of the dense form (endgame.hpp): the paths of systems the
// dense kernels tracked, f and J_f from their dense coefficient tables.
#include "endgame.hpp"

int hp::launch_endgame_dense(int n, const KArgs &a, const int2 *blk, int blocks, hipStream_t s) {
  return endgame_dispatch<DenseEndgame>(n, a, blk, blocks, s);
}
