"""Pins of the oracle's time bookkeeping and of the TP06 buffering root (CPU).

* Activation time (Sec. 3.3 uses the local activation time; the threshold
  crossing reading is the project's).  With no ionic current (linear model,
  g = 0) and a stimulus that covers every node from t = 0, each diffusion
  substep adds exactly dt_ad times the amplitude, so the potential sampled at
  reaction entry of outer step n is V0 + a (n + 1/2) dt: the continuous line
  V0 + a t sampled at t = (n + 1/2) dt.  Linear interpolation between two
  samples of a line is exact, so the recorded crossing must be
  (V_thr - V0)/a whatever dt, l and the threshold are.  Dating the sample at
  the start of the step (n dt) or at its end ((n + 1) dt), or interpolating
  from the wrong end, moves it by dt/2 or more.
* Stimulus window (Sec. 2: the stimulus enters step B; the reading is that a
  substep is stimulated when its start time tau has t_on <= tau < t_on + dur).
  With g = 0 and zero-flux boundaries the stiffness matrix has zero row and
  column sums, so the charge sum_i m_i V_i changes only through the stimulus:
  by a dt_ad sum_{i in stim} m_i per stimulated substep.  Substep starts are
  j dt_ad (j = 0, 1, ...) in exact arithmetic; with dt_ad a power of two and
  window edges that are exact binary fractions the number of stimulated
  substeps is a closed-form count, checked for windows that open and close on
  and between substep starts, on half-step and outer-step edges, shorter than
  one substep, and overlapping.
* Instantaneous buffering (TP06 calcium pools): the free concentration c
  carried by a total t solves t = c + B c / (c + K); the oracle's root is
  checked against that relation, against its inverse map, and against the
  limits B = 0 (c = t) and K -> 0 (c = max(t - B, 0)).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2011_04747_amd import workloads as W


def _cable(n, h=0.01, D=0.001):
    xyz, conn, et = W.structured_grid((n,), h)
    De = np.full((conn.shape[0], 1, 1), D)
    return W.Mesh(1, xyz, et, conn, De, grid_shape=(n,))


def _passive(o, V0):
    o.set_model(W.MODEL_LINEAR, np.vstack([np.zeros(o.n), np.zeros(o.n)]),
                init_state=np.full((1, o.n), V0), dt0=0.01, lat_threshold=o._thr)


@pytest.mark.parametrize("dt,V0,a,thr", [
    (0.1, -80.0, 3.7, -40.0),       # l = 2 on this cable
    (0.125, 0.0, 0.013, 0.37),      # dt_ad = 2^-5
    (0.05, -85.0, 11.0, -40.0),     # l = 1
    (0.1, 1.0, 0.5, 3.05),          # crossing exactly on a sample time: t* = 4.1 = 40.5 dt
    (0.2, -60.0, 0.9, -59.95),      # crossing inside the first sampled interval after step 0
])
def test_lat_is_the_crossing_time_of_a_linear_ramp(oracle_mod, dt, V0, a, thr):
    o = oracle_mod.Oracle(_cable(6))
    o._thr = thr
    _passive(o, V0)
    o.add_stimulus(np.arange(o.n), 0.0, 1e6, a)
    t_star = (thr - V0) / a
    n_steps = int(t_star / dt) + 3
    o.step(n_steps, dt)
    lat = o.get(oracle_mod.F_LAT)
    # the sampled potential itself is on the line (checks the dt/2 offset of
    # the sample independently of the interpolation)
    vb = o.get(oracle_mod.F_VPREV)
    np.testing.assert_allclose(vb, V0 + a * (n_steps - 0.5) * dt, rtol=0, atol=1e-11 * (1 + abs(V0)))
    if t_star < 0.5 * dt:
        # crossed before the first sample: no earlier sample to bracket it
        assert (lat < 0).all()
    else:
        np.testing.assert_allclose(lat, t_star, rtol=0, atol=1e-11 * max(1.0, t_star))


def _window_count(dt_ad, n_sub, t_on, dur):
    """Substep starts j dt_ad (j < n_sub) with t_on <= j dt_ad < t_on + dur, exactly."""
    d, a, b = Fr(dt_ad), Fr(t_on), Fr(t_on) + Fr(dur)
    return sum(1 for j in range(n_sub) if a <= j * d < b)


@pytest.mark.parametrize("windows", [
    [(0.0, 0.0625, 1.0)],                       # opens at t = 0, closes on a substep start
    [(0.03125, 0.03125, 1.0)],                  # exactly one substep, on its edges
    [(0.046875, 0.0625, 1.0)],                  # opens and closes between substep starts
    [(0.0625, 0.125, 1.0)],                     # opens on the half-step edge (the reaction)
    [(0.25, 0.0078125, 1.0)],                   # shorter than a substep, opens on an outer-step edge
    [(0.2578125, 0.0078125, 1.0)],              # shorter than a substep, between starts: none
    [(0.5, 1.0, 1.0), (0.75, 0.5, 2.5)],        # overlapping stimuli add
    [(0.0, 10.0, 1.0)],                         # longer than the run
])
def test_stimulated_substeps_match_the_closed_form_count(oracle_mod, windows):
    m = _cable(9)
    o = oracle_mod.Oracle(m)
    o._thr = 1e9
    _passive(o, 0.0)
    dt = 0.125
    o.prepare(dt)
    inf = o.info()
    l, dt_ad = inf["l"], inf["dt_ad"]
    assert (l, dt_ad) == (2, 0.03125)     # G = 4 D / h^2 = 40 on this cable
    stim = np.array([0, 1, 2, 7], np.int32)
    for (t_on, dur, amp) in windows:
        o.add_stimulus(stim, t_on, dur, amp)
    mass = o.matrix()[3]
    n_steps = 12
    o.step(n_steps, dt)
    q = float(np.dot(mass, o.get(oracle_mod.F_V)))
    n_sub = 2 * l * n_steps
    expect = sum(amp * dt_ad * mass[stim].sum() * _window_count(dt_ad, n_sub, t_on, dur)
                 for (t_on, dur, amp) in windows)
    # one stimulated substep adds about 3e-4 of charge here: an off-by-one
    # count is 1e8 times the tolerance
    assert q == pytest.approx(expect, rel=1e-12, abs=1e-15)


# published buffer constants of the three TP06 calcium pools (B mM, K mM)
_POOLS = [(0.2, 0.001), (0.4, 0.00025), (10.0, 0.3)]


@pytest.mark.parametrize("B,K", _POOLS + [(1.0, 1.0), (3.0, 1e-6)])
def test_buffer_root_solves_its_defining_relation(oracle_mod, B, K):
    rng = np.random.default_rng(7)
    # free concentrations over the physiological range and beyond
    for c in np.concatenate([10.0 ** rng.uniform(-7, 1.5, 200), [0.0]]):
        t = c + B * c / (c + K)                     # total that carries c
        c_hat = oracle_mod.buffer_free_from_total(t, B, K)
        # the root -b/2 + sqrt(b^2/4 + K t) with b = B + K - t loses digits to
        # cancellation when |b| >> c, and t itself carries a rounding of a few
        # ulps: the absolute error is a few ulps of |b| + t
        tol = 16 * np.finfo(float).eps * (abs(B + K - t) + c + t)
        assert abs(c_hat - c) <= tol, (c, c_hat, tol)
        assert c_hat >= 0.0
        # and the oracle's own forward map sends it back
        t_hat = oracle_mod.buffer_total_from_free(c_hat, B, K)
        assert abs(t_hat - t) <= tol * (1 + B / K) + 4 * np.finfo(float).eps * t


def test_buffer_root_limits(oracle_mod):
    for t in [0.0, 1e-6, 0.3, 2.0, 17.0]:
        # no buffer: free = total (to the cancellation bound of the root)
        eps16 = 16 * np.finfo(float).eps
        assert abs(oracle_mod.buffer_free_from_total(t, 0.0, 0.5) - t) <= eps16 * (abs(0.5 - t) + t)
        # a buffer that binds at any concentration (K -> 0) takes the first B
        c = oracle_mod.buffer_free_from_total(t, 1.0, 1e-12)
        assert c == pytest.approx(max(t - 1.0, 0.0), abs=1e-9)
    # small totals: the buffer is linear, c = t / (1 + B/K)
    for B, K in _POOLS:
        t = 1e-9 * K
        assert oracle_mod.buffer_free_from_total(t, B, K) == pytest.approx(t / (1 + B / K), rel=1e-6)
