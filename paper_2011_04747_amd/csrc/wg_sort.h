// Stable counting sort of a workgroup's nodes by a small key, in LDS (device
// code): the reaction kernels process nodes in order of their substep count
// so that a wavefront mixes counts only where two keys meet.
#pragma once
#include <hip/hip_runtime.h>

namespace mono {

// Key q in [0, NK) of this lane's node, or q < 0 for no node.  On return
// slot_node[t] holds the lane (workgroup-local node) whose node is t-th in
// key order, for t below the number of lanes with a node.  Every lane of the
// workgroup must call it (it contains barriers).
template <int BLOCK, int NK>
__device__ __forceinline__ void wg_order_by_key(int q, int* slot_node) {
  constexpr int W = BLOCK / 64;
  __shared__ int wcount[NK][W];   // nodes of key q in wavefront w, then their start
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long mine = 0ull;
  for (int kk = 0; kk < NK; ++kk) {
    const unsigned long long m = __ballot(q == kk);
    if (q == kk) mine = m;
    if (lane == 0) wcount[kk][w] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int kk = 0; kk < NK; ++kk)
      for (int v = 0; v < W; ++v) {
        const int c = wcount[kk][v];
        wcount[kk][v] = run;
        run += c;
      }
  }
  __syncthreads();
  if (q >= 0) slot_node[wcount[q][w] + __popcll(mine & ((1ull << lane) - 1ull))] = threadIdx.x;
  __syncthreads();
}

}  // namespace mono
