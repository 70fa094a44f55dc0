"""Edge cases of the boundary: empty work and empty inputs.

* Zero outer steps (graph, eager and timed modes) change nothing, a negative
  count is EINVAL.
* A stimulus with no nodes, or with a window of zero length (t_on <= tau <
  t_on + 0 holds for no substep start), adds nothing: the same bits as the
  simulation without it.  The ninth stimulus is EUNSUPPORTED, a node out of
  range or a negative duration EINVAL.
* An adjoint run with no sensors has a zero loss, and its backward sweep
  (no adjoint source anywhere) gives gradients that are exactly zero.
"""
import numpy as np
import pytest

from paper_2011_04747_amd import mono
from paper_2011_04747_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    T.cuda.set_device(0)
    return T


def _fields(s):
    S = s.info()["n_states"]
    return [s.get(mono.FIELD_V), s.get(mono.FIELD_VPREV), s.get(mono.FIELD_LAT)] + \
        [s.state(j) for j in range(1, S)]


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_zero_steps_change_nothing(torch, prec):
    w = W.slab_ischemic(shape=(13, 11, 7), t_end=2.0)
    s = mono.Sim.from_workload(w, prec)
    s.step(7, w.dt)
    before, step0 = _fields(s), s.info()["step"]
    for flags in (0, mono.STEP_EAGER, mono.STEP_TIMED):
        s.step(0, w.dt, flags=flags)
        s.sync()
        assert s.info()["step"] == step0
        _same(before, _fields(s))
    with pytest.raises(mono.MonoError) as e:
        s.step(-1, w.dt)
    assert mono.STATUS[e.value.code] == "EINVAL"
    s.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_empty_and_zero_length_stimuli_add_nothing(torch, prec):
    w = W.sheet_tp06(n=23, t_end=4.0)
    ref = mono.Sim.from_workload(w, prec)
    s = mono.Sim.from_workload(w, prec)
    s.add_stimulus(np.zeros(0, np.int32), 0.0, 2.0, 100.0)
    s.add_stimulus(np.arange(w.mesh.n_nodes, dtype=np.int32), 1.0, 0.0, 100.0)
    for x in (ref, s):
        x.step(w.n_steps, w.dt)
    _same(_fields(ref), _fields(s))
    ref.close()
    s.close()


def test_stimulus_arguments_are_checked(torch):
    w = W.sheet_tp06(n=9, t_end=1.0)
    s = mono.Sim.from_workload(w, "f64")
    nodes = np.arange(3, dtype=np.int32)
    for bad in (dict(nodes=np.array([w.mesh.n_nodes], np.int32), t_on=0.0, duration=1.0),
                dict(nodes=np.array([-1], np.int32), t_on=0.0, duration=1.0),
                dict(nodes=nodes, t_on=0.0, duration=-1.0),
                dict(nodes=nodes, t_on=float("nan"), duration=1.0)):
        with pytest.raises(mono.MonoError) as e:
            s.add_stimulus(bad["nodes"], bad["t_on"], bad["duration"], 10.0)
        assert mono.STATUS[e.value.code] == "EINVAL"
    n0 = len(w.stimuli)
    for q in range(8 - n0):
        s.add_stimulus(nodes, 0.0, 1.0, 10.0)
    with pytest.raises(mono.MonoError) as e:
        s.add_stimulus(nodes, 0.0, 1.0, 10.0)
    assert mono.STATUS[e.value.code] == "EUNSUPPORTED"
    s.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adjoint_without_sensors_is_zero(torch, prec):
    w = W.adjoint_slab(shape=(11, 9, 5), t_end=3.0, n_sensors=8)
    s = mono.Sim.from_workload(w, prec)
    s.set_sensors(np.zeros(0, np.int32), np.zeros((w.n_steps, 0)))
    loss = s.forward_taped(w.n_steps, w.dt, 7)
    gs, gp = s.backward()
    assert loss == 0.0
    assert not np.any(gs) and not np.any(gp)
    s.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_forced_unstable_diffusion_latches(torch, prec):
    """Failure injection from the host: l forced below the Gershgorin bound
    of eq. 3 makes the explicit diffusion unstable, the potential grows
    without bound, turns non-finite and the simulation latches (ENONFINITE at
    the next synchronising call, ESTATE for further steps), the same chain
    as a non-finite state set directly.  The same run at its own l stays
    finite."""
    w = W.slab_ischemic(shape=(21, 19, 9), t_end=60.0)
    rng = np.random.default_rng(5)
    ok = mono.Sim.from_workload(w, prec)
    ok.prepare(w.dt)
    assert ok.info()["l"] >= 3
    v0 = ok.get(mono.FIELD_V) + rng.uniform(-1.0, 1.0, w.mesh.n_nodes)
    ok.set(mono.FIELD_V, v0)
    ok.step(300, w.dt)
    ok.sync()
    assert np.isfinite(ok.get(mono.FIELD_V)).all()
    ok.close()
    s = mono.Sim.from_workload(w, prec)
    s.set(mono.FIELD_V, v0)
    s.force_l(1)
    with pytest.raises(mono.MonoError) as e:
        for _ in range(60):
            s.step(10, w.dt)
            s.sync()
    assert mono.STATUS[e.value.code] == "ENONFINITE"
    with pytest.raises(mono.MonoError) as e:
        s.step(1, w.dt)
    assert mono.STATUS[e.value.code] == "ESTATE"
    s.close()
