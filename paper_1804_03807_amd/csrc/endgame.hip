// End game kernels of the term form, the selection of the paths the end
// game refines, and the launcher of both forms (endgame.hpp).
#include "endgame.hpp"

namespace hp {
namespace {

// The queue indices whose paths the end game refines, compacted per system
// (from the system's eg_list_base) with one atomic per wavefront (ballot,
// popcount, mbcnt), so that the end game's wavefronts are full instead of
// one converged path among many stopped or suspended ones, and each still
// holds paths of one system.  Block b covers 64 queue entries of one
// system: blk[b] = (system, first index), or for one system (blk ==
// nullptr) indices 64 b .. 64 b + 63 of system 0.
__global__ void __launch_bounds__(64) k_eg_select(KArgs a, const int2 *blk, long long *list,
                                                  unsigned *counts) {
  const int lane = threadIdx.x & 63;
  int s = 0;
  long long q = (long long)blockIdx.x * 64 + lane;
  if (blk) {
    const int2 b = blk[blockIdx.x];
    s = b.x;
    q = (long long)b.y + lane;
  }
  cptr<DevSys> sp = as_const(a.sys) + s;
  bool take = false;
  if (q < sp->n_paths) {
    const long long *slots = (const long long *)sp->slots;
    const int st = a.status[sp->out_path_base + (slots ? slots[q] : q)];
    take = st == HP_CONVERGED || st == HP_FAILED_NEWTON_T1;
  }
  const uint64_t m = __ballot(take);
  if (m == 0) return;
  const int first = __builtin_ctzll(m);
  unsigned base = 0;
  if (lane == first) base = atomicAdd(counts + s, (unsigned)__popcll(m));
  base = __shfl(base, first);
  if (!take) return;
  list[sp->eg_list_base + base +
       __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = q;
}

}  // namespace
}  // namespace hp

int hp_launch_eg_select(const hp::KArgs &a, const int2 *blk, int blocks, long long *list,
                        unsigned *count, void *stream) {
  if (blocks <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(hp::k_eg_select, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)stream, a,
                     blk, list, count);
  return (int)hipGetLastError();
}

int hp_launch_endgame(int n, const hp::KArgs &a, const int2 *blk, int blocks, bool dense,
                      void *stream) {
  using namespace hp;
  if (blocks <= 0) return (int)hipSuccess;
  hipStream_t s = (hipStream_t)stream;
  if (dense) return launch_endgame_dense(n, a, blk, blocks, s);
  return endgame_dispatch<Endgame>(n, a, blk, blocks, s);
}
