"""The entry point that allocates nothing (mono_sample_sensors_noalloc)
against the allocating mono_sample_sensors, through the C interface: the
same samples bit for bit on two calls in a row (the second smaller), the
static buffer's limit, and the prepared-dt requirement."""
import ctypes as C

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


def _sim(w, sensors, prec):
    s = mono.Sim.from_workload(w, prec)
    s.set_sensors(sensors, np.zeros((0, len(sensors))))
    return s


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_sampling_equals_allocating_sampling(torch, prec):
    w = W.slab_ischemic(shape=(23, 19, 9), t_end=20.0)
    rng = np.random.default_rng(21)
    sensors = np.sort(rng.choice(w.mesh.n_nodes, 300, replace=False)).astype(np.int32)
    a = _sim(w, sensors, prec)
    b = _sim(w, sensors, prec)
    a.prepare(w.dt)
    b.prepare(w.dt)
    # first call: 120 steps x 300 sensors; second: 40 steps (smaller), then a
    # third with fewer sensors
    for steps in (120, 40):
        ref = a.sample_sensors(steps, w.dt, len(sensors))
        got = np.zeros((steps, len(sensors)))
        rc = mono.lib().mono_sample_sensors_noalloc(b.h, C.c_int64(steps), C.c_double(w.dt),
                                                    got.ctypes.data)
        assert rc == 0, mono.lib().mono_last_error()
        assert np.array_equal(got, ref)
        assert a.info()["step"] == b.info()["step"]
    few = sensors[::7].copy()
    a.set_sensors(few, np.zeros((0, len(few))))
    b.set_sensors(few, np.zeros((0, len(few))))
    ref = a.sample_sensors(25, w.dt, len(few))
    got = b.sample_sensors_noalloc(25, w.dt, len(few))
    assert np.array_equal(got, ref)
    assert np.array_equal(a.get(mono.FIELD_V), b.get(mono.FIELD_V))
    a.close()
    b.close()


def test_noalloc_sampling_limits(torch):
    w = W.cable_ms(t_end=5.0)
    sensors = np.arange(0, 101, 2, dtype=np.int32)          # 51 sensors
    s = _sim(w, sensors, "f64")
    # dt not prepared yet: refused before anything runs
    with pytest.raises(mono.MonoError) as e:
        s.sample_sensors_noalloc(4, w.dt, len(sensors))
    assert e.value.code == -4
    s.prepare(w.dt)
    # 10281 steps x 51 sensors > 524288 samples: refused
    with pytest.raises(mono.MonoError) as e:
        s.sample_sensors_noalloc(10281, w.dt, len(sensors))
    assert e.value.code == -1
    assert s.info()["step"] == 0
    # at the limit: 10280 x 51 = 524280 samples
    out = s.sample_sensors_noalloc(10280, w.dt, len(sensors))
    assert out.shape == (10280, 51) and np.isfinite(out).all()
    s.close()
