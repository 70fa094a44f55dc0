"""Checkpoint and resume through the boundary: a snapshot of V, V_prev, the
activation times, every cell state and the time level, taken with
mono_get_state, written to a file and read back, restores a fresh simulation
of the same mesh (mono_set_state, mono_set_time_level) so that it continues
with the same bits as a run that never stopped: V, every state, the
activation times and the substep counts, through a stimulus window that opens
after the resume point, in FP32 and FP64, in graph and eager stepping."""
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
    f = {"V": s.get(mono.FIELD_V), "VPREV": s.get(mono.FIELD_VPREV),
         "LAT": s.get(mono.FIELD_LAT)}
    for j in range(1, S):
        f[f"S{j}"] = s.state(j)
    return f


def _restore(s, f, step):
    s.set(mono.FIELD_V, f["V"])
    s.set(mono.FIELD_VPREV, f["VPREV"])
    s.set(mono.FIELD_LAT, f["LAT"])
    for j in range(1, s.info()["n_states"]):
        s.set(mono.FIELD_STATE0 + j, f[f"S{j}"])
    s.set_time_level(step)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("flags", [0, mono.STEP_EAGER])
def test_resume_in_a_new_simulation_is_bitwise(torch, tmp_path, prec, flags):
    # S1 at t = 0, the cross-field S2 at 4 ms: the resume point (2.5 ms) lies
    # between them
    w = W.slab_ischemic(shape=(27, 23, 9), t_end=8.0, s2_time=4.0)
    n1, n2 = 25, w.n_steps - 25
    ref = mono.Sim.from_workload(w, prec)
    ref.step(n1 + n2, w.dt, flags=flags)
    want = _fields(ref)
    want_k = ref.get(mono.FIELD_K)
    ref.close()

    a = mono.Sim.from_workload(w, prec)
    a.step(n1, w.dt, flags=flags)
    step = a.info()["step"]
    np.savez(tmp_path / "snap.npz", step=step, **_fields(a))
    a.close()

    snap = np.load(tmp_path / "snap.npz")
    b = mono.Sim.from_workload(w, prec)
    _restore(b, {k: snap[k] for k in snap.files if k != "step"}, int(snap["step"]))
    assert b.info()["step"] == n1
    b.step(n2, w.dt, flags=flags)
    got = _fields(b)
    for k, v in want.items():
        assert np.array_equal(v, got[k]), k
    assert np.array_equal(want_k, b.get(mono.FIELD_K))
    assert (got["LAT"] > 0).any()
    b.close()
