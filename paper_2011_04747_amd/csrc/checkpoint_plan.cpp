// Binomial checkpoint plans (dynamic programming over recursive splits).
#include "checkpoint_plan.h"

#include <algorithm>
#include <limits>

namespace mono {

bool make_ckpt_plan(int64_t n, int slots, CkptPlan& p) {
  if (n < 1 || slots < 1 || (n > 1 && slots < 2)) return false;
  const int width = (int)std::min<int64_t>(slots, n);   // free slots 0 .. slots-1, capped
  if ((double)n * (double)n * (double)width > 2e9) return false;
  const int64_t INF = std::numeric_limits<int64_t>::max() / 4;
  p.n = n;
  p.slots = slots;
  p.width = width;
  const size_t sz = (size_t)(n + 1) * width;
  p.costF.assign(sz, INF);
  p.costA.assign(sz, INF);
  p.splitF.assign(sz, 0);
  p.splitA.assign(sz, 0);
  for (int f = 0; f < width; ++f) {
    p.costF[p.idx(1, f)] = 0;
    p.costA[p.idx(1, f)] = 0;
  }
  for (int64_t k = 2; k <= n; ++k) {
    for (int f = 0; f < width; ++f) {
      int64_t bf = INF, ba = INF;
      int32_t mf = 0, ma = 0;
      for (int64_t m = 1; m < k; ++m) {
        const int64_t left = p.costF[p.idx(m, f)];
        if (left >= INF) continue;
        // reverse the k - m segments after the split: a single one from the
        // live state, more from a stored state with one buffer fewer
        const int64_t right_f = (k - m == 1) ? 0 : (f >= 1 ? p.costF[p.idx(k - m, f - 1)] : INF);
        if (right_f < INF && m + right_f + left < bf) {
          bf = m + right_f + left;
          mf = (int32_t)m;
        }
        const int64_t right_a = f >= 1 ? p.costA[p.idx(k - m, f - 1)] : INF;
        if (right_a < INF && right_a + left < ba) {
          ba = right_a + left;
          ma = (int32_t)m;
        }
      }
      p.costF[p.idx(k, f)] = bf;
      p.splitF[p.idx(k, f)] = mf;
      // or the forward run stores nothing more here (split 0): recompute
      if (bf <= ba) {
        ba = bf;
        ma = 0;
      }
      p.costA[p.idx(k, f)] = ba;
      p.splitA[p.idx(k, f)] = ma;
    }
  }
  return p.costA[p.idx(n, width - 1)] < INF;
}

}  // namespace mono
