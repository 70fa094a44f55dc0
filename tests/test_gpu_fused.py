"""The fused half-step diffusion (up to four substeps of a half step per
launch on 3D structured grids) against the unfused launches, which the
parity tests hold to the FP64 CPU oracle.

Bar: the same bits.  Every node's update reads the same weights in the same
order as the one-substep kernels, so V, every state row, activation times
and substep counts must be equal element for element, in FP32 and FP64,
for l = 2 .. 8 (one or two fused launches per half step, chunks of unequal
length), z tiles of one plane up to the whole grid, grids whose sides are
not multiples of the tile (ragged x, y and z tails), stimulus windows that
open and close inside a fused launch, the stimulus-free graphs, and eager
stepping."""
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


def _slab(shape=(70, 37, 23), t_end=8.0):
    # S1 on x = 0 from t = 0, the cross-field S2 at 3 ms: both windows fall
    # inside the run
    return W.slab_ischemic(shape=shape, dx=2.0 ** -7, t_end=t_end, s2_time=3.0)


def _run(w, prec, l=None, flags=0, **launch):
    s = mono.Sim.from_workload(w, prec)
    if launch:
        s.set_launch(**launch)
    if l:
        s.force_l(l)
    s.step(w.n_steps, w.dt, flags=flags)
    S = s.info()["n_states"]
    out = [s.get(mono.FIELD_V), s.get(mono.FIELD_LAT), s.get(mono.FIELD_K),
           s.get(mono.FIELD_VPREV)] + [s.state(j) for j in range(1, S)]
    info = s.info()
    s.close()
    return out, info


def _same(a, b, what):
    for f, (x, y) in enumerate(zip(a, b)):
        bad = np.flatnonzero(x != y)
        assert bad.size == 0, (what, f, bad.size, bad[:5], x[bad[:5]], y[bad[:5]])


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("l", [2, 3, 4, 5, 8])
def test_fused_matches_unfused_bitwise(torch, prec, l):
    w = _slab()
    ref, info0 = _run(w, prec, l, diff_fuse=0)
    assert info0["diff_fused"] == 1 and info0["diff_launches"] == l
    for planes in (0, 1, 5, 23):
        out, info = _run(w, prec, l, diff_fuse=1, diff_fuse_planes=planes)
        assert info["l"] == l and info["diff_launches"] == (l + 3) // 4
        _same(ref, out, (prec, l, planes))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_eager_and_graph_sizes(torch, prec):
    """Eager launches and graphs of a few steps (stimulus-free graphs for the
    steps no window touches) give the bits of unfused stepping."""
    w = _slab(shape=(61, 17, 9), t_end=6.0)
    ref, _ = _run(w, prec, diff_fuse=0)
    out, info = _run(w, prec, flags=mono.STEP_EAGER, diff_fuse=1)
    assert info["diff_launches"] == (info["l"] + 3) // 4
    _same(ref, out, "eager")
    for g in (1, 7, 64):
        out, _ = _run(w, prec, graph_steps=g, diff_fuse=1)
        _same(ref, out, ("graph", g))


def test_fused_at_the_parity_test_shape(torch):
    """The slab at the sizes of the parity tests (default launch: unfused)
    and the fused kernel with the autotuner's plane choices, bitwise."""
    w = W.slab_ischemic(shape=(29, 23, 13), t_end=12.0)
    ref, info0 = _run(w, "f32")
    assert info0["diff_launches"] == info0["l"]
    for planes in (0, 2, 13):
        out, info = _run(w, "f32", diff_fuse=1, diff_fuse_planes=planes)
        assert info["diff_fused"] == 1
        _same(ref, out, planes)


def test_fused_only_where_the_grid_admits_it(torch):
    s = mono.Sim.from_workload(W.sheet_tp06(n=41), "f32")       # 2D grid
    s.prepare(0.1)
    assert s.info()["diff_fused"] == 0 and s.info()["diff_launches"] == s.info()["l"]
    s.close()
    s = mono.Sim.from_workload(W.batched_sheets(n_inst=3, side_lo=12, side_hi=20), "f32")
    assert s.info()["diff_fused"] == 0
    s.close()
    s = mono.Sim.from_workload(W.slab_ischemic_tets(shape=(9, 8, 5)), "f32")
    assert s.info()["diff_fused"] == 0
    s.close()
    # row classes off: the fused kernel reads rows by class, so it stays off
    w = _slab(shape=(30, 20, 8), t_end=1.0)
    s = mono.Sim.from_workload(w, "f32")
    s.set_launch(diff_classes=0, diff_fuse=1)
    s.prepare(w.dt)
    assert s.info()["diff_fused"] == 1 and s.info()["diff_launches"] == s.info()["l"]
    s.close()


def test_fused_diffusion_timing_leaves_the_potential_in_place(torch):
    """The diffusion timing hook runs whole fused half steps (an even number
    of launches), so the simulation steps on from a finite potential."""
    w = _slab(shape=(40, 20, 10), t_end=2.0)
    s = mono.Sim.from_workload(w, "f32")
    s.set_launch(diff_fuse=1)
    s.force_l(5)                                       # 2 launches per half step
    s.prepare(w.dt)
    ms = s.time_diffusion(10)
    assert ms > 0.0
    s.step(5, w.dt)
    assert np.isfinite(s.get(mono.FIELD_V)).all()
    s.close()


def test_launch_rejects_bad_fuse_fields(torch):
    s = mono.Sim.from_workload(_slab(shape=(20, 10, 6), t_end=1.0), "f32")
    for bad in (dict(diff_fuse=2), dict(diff_fuse=-1), dict(diff_fuse_planes=-1),
                dict(diff_fuse_planes=4097)):
        with pytest.raises(mono.MonoError):
            s.set_launch(**bad)
    s.close()
