"""Pins of the oracle's APD90 measurement (paper Sec. 4: APD90 measured from
the time of the maximum upstroke derivative) on sample sequences whose answer
is known in closed form, and its invariances."""
import numpy as np
import pytest

from oracle.oracle import apd90


def _trace():
    # dt = 1 ms, samples at t_n = n + 1/2.  Rest at -80 mV, upstroke over two
    # intervals (slopes 40 and 60 mV/ms), peak 30 mV at n = 7, then a linear
    # decay of 10 mV per sample.  Threshold -60: activation at n = 5
    # (V_rest = -80).  V_90 = 30 - 0.9 * 110 = -69, crossed between n = 16
    # (-60) and n = 17 (-70) at 9/10 of the interval: t = 16.5 + 0.9 = 17.4.
    # Steepest interval n = 6: midpoint 6.0.  APD90 = 11.4 ms.
    v = np.full(40, -80.0)
    v[5], v[6] = -40.0, 20.0
    for n in range(7, 40):
        v[n] = 30.0 - 10.0 * (n - 7)
    return v


def test_piecewise_linear_closed_form():
    a, t = apd90(_trace()[:, None], 1.0, -60.0)
    assert t[0] == pytest.approx(6.0, abs=1e-12)
    assert a[0] == pytest.approx(11.4, abs=1e-12)


def test_time_step_and_origin():
    # the same trace sampled with dt = 0.25 ms from step 100: every time
    # scales by dt and shifts by 100 dt
    v = _trace()
    a, t = apd90(v[:, None], 0.25, -60.0, step0=100)
    assert t[0] == pytest.approx(100 * 0.25 + 6.0 * 0.25, abs=1e-12)
    assert a[0] == pytest.approx(11.4 * 0.25, abs=1e-12)


def test_affine_voltage_map():
    # V -> 2 V + 5 with the threshold mapped alike leaves every time unchanged
    v = _trace()
    a0, t0 = apd90(v[:, None], 1.0, -60.0)
    a1, t1 = apd90((2.0 * v + 5.0)[:, None], 1.0, 2.0 * -60.0 + 5.0)
    assert t1[0] == pytest.approx(t0[0], abs=1e-12)
    assert a1[0] == pytest.approx(a0[0], abs=1e-12)


def test_first_action_potential_only_and_ties():
    v = _trace()
    # a second action potential after repolarisation changes nothing
    w = np.concatenate([v[:25], np.full(5, -80.0), v[:20]])
    a0, t0 = apd90(v[:, None], 1.0, -60.0)
    a1, t1 = apd90(w[:, None], 1.0, -60.0)
    assert (a1[0], t1[0]) == (a0[0], t0[0])
    # two equally steep intervals: the first one gives the upstroke time
    u = v.copy()
    u[5], u[6], u[7] = -20.0, 40.0, 45.0     # slopes 60, 60, 5
    _, t = apd90(u[:, None], 1.0, -60.0)
    assert t[0] == pytest.approx(5.0, abs=1e-12)


def test_unmeasured_nodes():
    rest = np.full(30, -80.0)
    plateau = _trace()[:12]                 # activates, never repolarises
    below = -61.0 + 0.0 * rest              # never reaches the threshold
    a, t = apd90(np.stack([rest, np.pad(plateau, (0, 18), constant_values=25.0), below], 1),
                 1.0, -60.0)
    assert a[0] == -1.0 and t[0] == -1.0
    assert a[1] == -1.0 and t[1] == pytest.approx(6.0, abs=1e-12)
    assert a[2] == -1.0 and t[2] == -1.0


def test_peak_taken_before_the_crossing():
    # V_90 follows the running maximum: a dip right after the first peak is
    # tested against the level of that peak (no crossing), although it lies
    # below the level of the later, higher peak
    v = np.full(40, -80.0)
    v[5] = 10.0                   # steepest interval (90 mV/ms); running V_90 = 10 - 0.9 * 90 = -71
    v[6] = -70.5                  # above -71: no repolarisation
    v[7] = 18.0                   # slope 88.5; peak 18: V_90 = 18 - 0.9 * 98 = -70.2
    for n in range(8, 40):
        v[n] = 18.0 - 10.0 * (n - 7)
    a, t = apd90(v[:, None], 1.0, -60.0)
    # crossing of -70.2 between n = 15 (-62) and n = 16 (-72): w = 0.82,
    # t_rep = 15.5 + 0.82; upstroke: midpoint of interval 5, 5.0
    assert t[0] == pytest.approx(5.0, abs=1e-12)
    assert a[0] == pytest.approx(15.5 + 0.82 - 5.0, abs=1e-9)
