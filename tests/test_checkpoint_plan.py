"""The binomial checkpoint plan of the adjoint's reverse sweep (host code,
no GPU), pinned by an exhaustive search over every schedule on small cases
and by the closed form of binomial checkpointing.

Model of a schedule: a run of n segments whose starts are positions
0 .. n-1.  The taped forward run passes every position once and may store
the state at any of them (free).  The reverse sweep then reverses segment
n-1, n-2, ..., 0; reversing segment j needs the state at position j, either
stored or the live state.  Between reversals the live state may be loaded
from a stored position (free), advanced by one segment (cost 1), stored
(at most `slots` stored states at a time) or dropped.  The plan's advance
count must equal the minimum over all such schedules.
"""
from collections import deque
from math import comb

import pytest

from paper_2011_04747_amd import mono


def _min_advances(n, slots):
    """Exhaustive 0-1 breadth-first search over schedule states
    (j, stored positions, live position)."""
    INF = float("inf")
    best = {}
    dq = deque()
    # the forward sweep stores any subset of at most `slots` positions
    for mask in range(1 << n):
        if bin(mask).count("1") <= slots:
            st = (n - 1, mask, -1)
            best[st] = 0
            dq.append((0, st))
    while dq:
        d, (j, mask, live) = dq.popleft()
        if d > best.get((j, mask, live), INF):
            continue
        if j < 0:
            return d
        nxt = []
        # reverse segment j from the live state or a stored one
        if live == j or (mask >> j) & 1:
            keep = mask & ((1 << j) - 1)           # positions after j are no longer needed
            nxt.append((0, (j - 1, keep, -1)))
        # load a stored position into the live state
        for p in range(j + 1):
            if (mask >> p) & 1 and p != live:
                nxt.append((0, (j, mask, p)))
        # store the live state
        if live >= 0 and not (mask >> live) & 1 and bin(mask).count("1") < slots:
            nxt.append((0, (j, mask | (1 << live), live)))
        # drop a stored position
        for p in range(j + 1):
            if (mask >> p) & 1:
                nxt.append((0, (j, mask & ~(1 << p), live)))
        # advance the live state by one segment
        if 0 <= live < j:
            nxt.append((1, (j, mask, live + 1)))
        for w, st in nxt:
            nd = d + w
            if nd < best.get(st, INF):
                best[st] = nd
                if w == 0:
                    dq.appendleft((nd, st))
                else:
                    dq.append((nd, st))
    raise AssertionError("no schedule")


@pytest.mark.parametrize("n", range(1, 9))
def test_plan_is_the_minimum_over_all_schedules(n):
    for slots in range(2, n + 2):
        got = mono.checkpoint_plan_advances(n, slots)
        assert got == _min_advances(n, slots), (n, slots)


def test_plan_extremes():
    for n in (1, 2, 7, 60, 300):
        # a buffer per segment start: the uniform schedule, no advances
        assert mono.checkpoint_plan_advances(n, n) == 0
        assert mono.checkpoint_plan_advances(n, n + 5) == 0
    for n in (9, 10, 11):
        # few buffers on longer runs, where most states are recomputed
        for slots in (2, 3):
            assert mono.checkpoint_plan_advances(n, slots) == _min_advances(n, slots)
    with pytest.raises(mono.MonoError):
        mono.checkpoint_plan_advances(5, 1)


def test_plan_reaches_the_binomial_bound():
    """With s buffers besides the run's start and r passes over the stored
    states, at most C(s + r, s) segments can be reversed (binomial
    checkpointing).  Here: beyond the taped run, each further pass over a
    segment is one advance, so n = C(s + r, s) segments need at most
    (r - 1) n advances, and one segment more needs more than the plan for n
    plus one."""
    for s in (1, 2, 3, 5):
        for r in (1, 2, 3):
            n = comb(s + r, s)
            a = mono.checkpoint_plan_advances(n, s + 1)
            assert a <= (r - 1) * n, (s, r, n, a)
            if n + 1 <= 400:
                assert mono.checkpoint_plan_advances(n + 1, s + 1) >= a
    # advances fall as buffers are added
    prev = None
    for slots in range(2, 61):
        a = mono.checkpoint_plan_advances(60, slots)
        if prev is not None:
            assert a <= prev
        prev = a
    assert prev == 0
