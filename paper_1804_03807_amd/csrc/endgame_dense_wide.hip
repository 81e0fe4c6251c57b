// End game kernels of the dense form (endgame.hpp) for n = 11 and 12.
#include "endgame.hpp"

int hp::launch_endgame_dense_wide(int n, const KArgs &a, const int2 *blk, int blocks,
                                  hipStream_t s) {
  switch (n) {
    case 11: return endgame_launch<11, DenseEndgame<11>>(a, blk, blocks, s);
    case 12: return endgame_launch<12, DenseEndgame<12>>(a, blk, blocks, s);
    default: return (int)hipErrorInvalidValue;
  }
}
