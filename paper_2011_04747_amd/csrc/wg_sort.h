// Stable counting sort of a workgroup's nodes by a small key, in LDS (device
// code): the reaction kernels process nodes in order of their substep count
// so that a wavefront mixes counts only where two keys meet.
#pragma once
#include <hip/hip_runtime.h>

namespace mono {

// Key q in [0, nk) of this lane's node (nk <= NK, uniform), or q < 0 for no
// node.  Returns false when the workgroup's nodes share one key: the order
// is then the identity and slot_node is not written.  Otherwise slot_node[t]
// holds the lane (workgroup-local node) whose node is t-th in key order, for
// t below the number of lanes with a node.  Every lane of the workgroup must
// call it (it contains barriers); the result is uniform.
template <int BLOCK, int NK>
__device__ __forceinline__ bool wg_order_by_key(int q, int nk, int* slot_node) {
  constexpr int W = BLOCK / 64;
  constexpr int NE = NK * W;                 // counts, key-major: [key * W + wavefront]
  constexpr int C = (NE + 63) / 64;          // entries per lane of the scanning wavefront
  __shared__ int wcount[NE];
  __shared__ unsigned int wkeys[W];          // keys present in each wavefront (bit per key)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long mine = 0ull;
  unsigned int present = 0u;
  for (int kk = 0; kk < nk; ++kk) {
    const unsigned long long m = __ballot(q == kk);
    if (q == kk) mine = m;
    if (m) present |= 1u << kk;
    if (lane == 0) wcount[kk * W + w] = __popcll(m);
  }
  if (lane == 0) wkeys[w] = present;
  __syncthreads();
  unsigned int all = 0u;
  for (int v = 0; v < W; ++v) all |= wkeys[v];
  if ((all & (all - 1u)) == 0u) return false;   // one key (or none): identity order
  if (w == 0) {
    // exclusive scan of the counts in key-major order: each lane sums a run
    // of C entries, the wavefront scans the run sums, each lane writes its
    // run's starts
    int cnt[C];
    int sum = 0;
    for (int c = 0; c < C; ++c) {
      const int e = lane * C + c;
      cnt[c] = (e < nk * W) ? wcount[e] : 0;
      sum += cnt[c];
    }
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    int run = incl - sum;
    for (int c = 0; c < C; ++c) {
      const int e = lane * C + c;
      if (e < nk * W) wcount[e] = run;
      run += cnt[c];
    }
  }
  __syncthreads();
  if (q >= 0) slot_node[wcount[q * W + w] + __popcll(mine & ((1ull << lane) - 1ull))] = threadIdx.x;
  __syncthreads();
  return true;
}

}  // namespace mono
