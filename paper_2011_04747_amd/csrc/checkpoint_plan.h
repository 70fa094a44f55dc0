// Binomial (revolve-type) checkpoint schedules for the adjoint's reverse sweep.
//
// The taped run is cut into n segments of ckpt_every outer steps.  The
// reverse sweep reverses segments from the last to the first; reversing
// segment j needs the state at its start, either in one of `slots` snapshot
// buffers (the run's initial state takes one) or as the simulation's live
// state (which the reversal then overwrites).  With fewer buffers than
// segments, the states in between are recomputed by forward advances of
// whole segments from an earlier snapshot.  The plan minimises the number
// of those advances by dynamic programming over the split point of each
// recursion:
//
//   F(1, f) = 0,
//   F(k, f) = min_{1 <= m < k}  m + R(k - m, f) + F(m, f),
//   R(1, f) = 0 (the last segment reversed from the live state),
//   R(j, f) = F(j, f - 1) for j > 1 (its start stored; needs f >= 1),
//
// reverses k segments whose first start is stored, with f further free
// buffers: advance m segments, reverse the k - m segments after them (from a
// stored state, with one buffer fewer, unless a single segment is left),
// then the first m with the buffer back.  The taped forward run passes every
// segment anyway, so the states its first splits need are stored on the way
// at no extra cost (the run's end state is not a segment start, so nothing
// is reversed from the live state there):
//
//   A(1, f) = 0,
//   A(k, f) = min( F(k, f), min_m  A(k - m, f - 1) + F(m, f) (f >= 1) ),
//
// the first option (split 0) storing nothing more on the way.
//
// With a buffer per segment this is the uniform schedule (no advances);
// with two buffers the plan is that of binomial checkpointing with a
// single stored state besides the start.  The minimum over such recursive
// splits is that of binomial checkpointing (Griewank and Walther's revolve);
// the tests compare it with an exhaustive search over all schedules.
#pragma once
#include <cstdint>
#include <vector>

namespace mono {

struct CkptPlan {
  int64_t n = 0;        // segments
  int slots = 0;        // snapshot buffers (the run's start included)
  int width = 0;        // free-slot values stored per k: 0 .. width-1
  std::vector<int64_t> costF, costA;
  std::vector<int32_t> splitF, splitA;
  int64_t idx(int64_t k, int f) const { return k * width + f; }
  // advances of the whole reverse sweep (after the taped forward run)
  int64_t advances() const { return costA[idx(n, width - 1)]; }
};

// Plan for n segments and `slots` buffers (2 <= slots, or n == 1).  Returns
// false when the table would be too large (n * n * slots above ~2e9).
bool make_ckpt_plan(int64_t n, int slots, CkptPlan& out);

}  // namespace mono
