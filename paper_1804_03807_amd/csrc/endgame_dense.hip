// End game kernels of the dense form (endgame.hpp) for n <= 10: the paths of
// systems the dense kernels tracked, f and J_f from their dense coefficient
// tables.  n = 11 and 12 sit in endgame_dense_wide.hip, a translation unit
// of their own so that the largest instantiations compile side by side.
#include "endgame.hpp"

int hp::launch_endgame_dense(int n, const KArgs &a, const int2 *blk, int blocks, hipStream_t s) {
  switch (n) {
    case 1: return endgame_launch<1, DenseEndgame<1>>(a, blk, blocks, s);
    case 2: return endgame_launch<2, DenseEndgame<2>>(a, blk, blocks, s);
    case 3: return endgame_launch<3, DenseEndgame<3>>(a, blk, blocks, s);
    case 4: return endgame_launch<4, DenseEndgame<4>>(a, blk, blocks, s);
    case 5: return endgame_launch<5, DenseEndgame<5>>(a, blk, blocks, s);
    case 6: return endgame_launch<6, DenseEndgame<6>>(a, blk, blocks, s);
    case 7: return endgame_launch<7, DenseEndgame<7>>(a, blk, blocks, s);
    case 8: return endgame_launch<8, DenseEndgame<8>>(a, blk, blocks, s);
    case 9: return endgame_launch<9, DenseEndgame<9>>(a, blk, blocks, s);
    case 10: return endgame_launch<10, DenseEndgame<10>>(a, blk, blocks, s);
    default: return launch_endgame_dense_wide(n, a, blk, blocks, s);
  }
}
