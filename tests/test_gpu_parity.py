"""Parity of the HIP path (through the C interface) with the FP64 CPU oracle.

Tolerances:
  * FP64: ||V_gpu - V_orc||_inf <= 1e-9 * max(||V_orc||_inf, V_ref) at every
    compared time level (V_ref = 1 for Mitchell-Schaeffer, 100 mV for TP06).
  * FP32: V RMS <= 0.5 mV over nodes and compared levels, max |dLAT| <= 0.5 ms
    over nodes activated in both runs, identical activated sets.
  * Integer decisions (k, l, k_max) bit-exact; where the GPU's own k differs
    from the oracle's, the oracle's dV/dt must lie within rounding of a
    decision boundary of the k rule (0 or an integer), since both outcomes
    are valid DAETI results there.  The GPU replays the oracle's k-trace so
    that such flips do not contaminate the state comparison.
"""
import math

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


def _oracle(w, **kw):
    from oracle.oracle import Oracle
    return Oracle.from_workload(w, **kw)


def _vref(w):
    return 100.0 if w.model == W.MODEL_TP06 else 1.0


def _check_flips(w, k_orc, d_orc, k_gpu):
    diff = k_orc != k_gpu
    nflip = int(diff.sum())
    if nflip:
        d = np.abs(d_orc[diff])
        dist = np.abs(d - np.rint(d))
        tol = 1e-9 * _vref(w) / w.dt
        assert (dist <= tol).all(), (nflip, d[dist > tol][:5])
    return nflip


def run_pair(torch, w, n_steps, precision="f64", layout=mono.LAYOUT_AUTO, every=None,
             replay=True, launch=None):
    """Run the oracle (recording its k decisions), then the GPU replaying them;
    returns per-level (V_orc, V_gpu), both simulations and the flip count."""
    o = _oracle(w)
    kt, dtr = o.record_k(n_steps, with_d=True)
    every = every or n_steps
    chunks = [min(every, n_steps - d) for d in range(0, n_steps, every)]
    vo = []
    for c in chunks:
        o.step(c, w.dt)
        vo.append(o.get(0))
    s = mono.Sim.from_workload(w, precision, layout=layout)
    if launch:
        s.set_launch(**launch)
    rep = torch.from_numpy(kt).cuda()
    rec = torch.zeros_like(rep)
    s.ktrace(3 if replay else 1, rec.data_ptr(), rep.data_ptr(), n_steps, 0)
    levels = []
    for c, v in zip(chunks, vo):
        s.step(c, w.dt)
        levels.append((v, s.get(mono.FIELD_V)))
    torch.cuda.synchronize()
    nflip = _check_flips(w, kt, dtr, rec.cpu().numpy())
    return o, s, levels, nflip


def _assert_f64_levels(w, levels):
    for vo, vg in levels:
        scale = max(np.abs(vo).max(), _vref(w))
        err = np.abs(vg - vo).max() / scale
        assert err <= 1e-9, err


# ---------------------------------------------------------------------------
# setup: eq. (3), l, k_max, lambda_max
# ---------------------------------------------------------------------------
def _meshes():
    sheet = W.sheet_tp06(n=41).mesh
    slab = W.slab_ischemic(shape=(21, 17, 11)).mesh
    cable = W.cable_ms().mesh
    batch = W.batched_sheets(n_inst=4, side_lo=12, side_hi=30).mesh
    return {"cable": cable, "sheet": sheet, "slab": slab, "batch": batch}


@pytest.mark.parametrize("name", ["cable", "sheet", "slab", "batch"])
@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_gershgorin_l_kmax_match_oracle(torch, name, layout):
    from oracle.oracle import Oracle
    m = _meshes()[name]
    o = Oracle(m)
    o.set_model(W.MODEL_LINEAR, np.vstack([np.zeros(m.n_nodes), np.zeros(m.n_nodes)]))
    o.prepare(0.1)
    s = mono.Sim(m, "f64", layout=layout)
    s.set_cell_model(W.MODEL_LINEAR, np.vstack([np.zeros(m.n_nodes), np.zeros(m.n_nodes)]))
    s.prepare(0.1)
    for q in range(m.n_instances):
        a, b = o.info(q), s.info(q)
        assert b["dt_s"] == pytest.approx(a["dt_s"], rel=1e-13)
        assert b["G_max"] == pytest.approx(a["G_max"], rel=1e-13)
        assert b["l"] == a["l"] and b["k_max"] == a["k_max"]
        assert b["dt_ad"] == a["dt_ad"]
        assert b["layout"] == layout


@pytest.mark.parametrize("name", ["sheet", "slab", "batch"])
def test_power_iteration_lambda(torch, name):
    from oracle.oracle import Oracle
    m = _meshes()[name] if name != "sheet" else W.sheet_tp06(n=21).mesh
    if name == "slab":
        m = W.slab_ischemic(shape=(9, 8, 7)).mesh
    if name == "batch":
        m = W.batched_sheets(n_inst=3, side_lo=8, side_hi=14).mesh
    o = Oracle(m)
    K, mass = o.dense_K()
    s = mono.Sim(m, "f64")
    s.set_cell_model(W.MODEL_LINEAR)
    s.prepare(0.1)
    s.estimate_lambda(400)
    off = m.inst_node_off if m.inst_node_off is not None else [0, m.n_nodes]
    for q in range(m.n_instances):
        sl = slice(off[q], off[q + 1])
        Ms = 1 / np.sqrt(mass[sl])
        lmax = np.linalg.eigvalsh(Ms[:, None] * K[sl, sl] * Ms[None, :]).max()
        inf = s.info(q)
        assert inf["lambda_est"] <= lmax * (1 + 1e-10)
        assert inf["lambda_est"] >= 0.8 * lmax
        assert inf["G_max"] >= lmax * (1 - 1e-12)
        assert inf["dt_ad"] < 2.0 / lmax


# ---------------------------------------------------------------------------
# diffusion closed forms and invariants on the GPU
# ---------------------------------------------------------------------------
def _cos_mode(shape, js):
    n = int(np.prod(shape))
    idx = np.arange(n)
    phi = np.ones(n)
    stride = 1
    for a in range(len(shape)):
        ia = (idx // stride) % shape[a]
        phi *= np.cos(math.pi * js[a] * ia / (shape[a] - 1))
        stride *= shape[a]
    return phi


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
@pytest.mark.parametrize("shape,hs,Ds,js", [
    ((301,), (0.01,), (0.001,), (7,)),
    ((37, 29), (0.01, 0.012), (0.0012, 0.0003), (2, 5)),
    ((13, 11, 9), (0.01, 0.01, 0.01), (0.0012, 0.0003, 0.0003), (4, 1, 2)),
])
def test_diffusion_cosine_mode_closed_form(torch, prec, layout, shape, hs, Ds, js):
    xyz, conn, et = W.structured_grid(shape, hs)
    d = len(shape)
    De = np.broadcast_to(np.diag(Ds)[None], (conn.shape[0], d, d)).copy()
    m = W.Mesh(d, xyz, et, conn, De)
    lam = 0.0
    for a in range(d):
        t = 2 * Ds[a] / hs[a] ** 2 * (1 - math.cos(math.pi * js[a] / (shape[a] - 1)))
        for b in range(d):
            if b != a:
                t *= (2 + math.cos(math.pi * js[b] / (shape[b] - 1))) / 3
        lam += t
    s = mono.Sim(m, prec, layout=layout)
    s.set_cell_model(W.MODEL_LINEAR, np.zeros((2, m.n_nodes)))
    phi = _cos_mode(shape, js)
    s.set(mono.FIELD_V, phi)
    s.step(9, 0.1)
    inf = s.info()
    amp = (1 - inf["dt_ad"] * lam) ** (2 * inf["l"] * 9)
    tol = 1e-12 if prec == "f64" else 2e-5
    assert np.abs(s.get(mono.FIELD_V) - amp * phi).max() <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_constant_potential_is_fixed_bitwise(torch, prec, layout):
    m = W.slab_ischemic(shape=(17, 13, 9)).mesh
    s = mono.Sim(m, prec, layout=layout)
    s.set_cell_model(W.MODEL_LINEAR, np.zeros((2, m.n_nodes)))
    c = -84.5
    s.set(mono.FIELD_V, np.full(m.n_nodes, c))
    s.step(40, 0.1)
    assert (s.get(mono.FIELD_V) == c).all()


def test_charge_conservation_fp64(torch):
    from oracle.oracle import Oracle
    m = W.batched_sheets(n_inst=3, side_lo=20, side_hi=40).mesh
    mass = Oracle(m).matrix()[3]
    s = mono.Sim(m, "f64")
    s.set_cell_model(W.MODEL_LINEAR, np.zeros((2, m.n_nodes)))
    V0 = np.random.default_rng(1).uniform(-80, 20, m.n_nodes)
    s.set(mono.FIELD_V, V0)
    s.step(50, 0.1)
    V = s.get(mono.FIELD_V)
    off = m.inst_node_off
    for q in range(3):
        sl = slice(off[q], off[q + 1])
        assert np.dot(mass[sl], V[sl]) == pytest.approx(np.dot(mass[sl], V0[sl]), rel=1e-13)


# ---------------------------------------------------------------------------
# whole-path parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_cable_ms_fp64_parity(torch, layout):
    w = W.cable_ms()                                   # 101 nodes, 100 ms
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, layout=layout, every=100)
    _assert_f64_levels(w, levels)
    assert np.abs(s.state(1) - o.state(1)).max() <= 1e-9
    lo, lg = o.get(2), s.get(mono.FIELD_LAT)
    assert ((lo > 0) == (lg > 0)).all() and (lo > 0).all()
    assert np.abs(lo - lg).max() <= 1e-9 * 100
    assert nflip <= 2


def test_cable_ms_fp64_free_running(torch):
    """Without k replay: the GPU and the oracle take their own k decisions."""
    w = W.cable_ms()
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, every=100, replay=False)
    if nflip == 0:
        _assert_f64_levels(w, levels)
    assert (s.get(mono.FIELD_LAT) > 0).all()


@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_sheet_tp06_fp64_parity(torch, layout):
    w = W.sheet_tp06(n=57, t_end=60.0)                 # 3249 nodes: 12.7 tiles
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, layout=layout, every=150)
    _assert_f64_levels(w, levels)
    for j in (1, 2, 3, 4, 5, 6, 7, 8, 12, 15, 16, 18):
        a, b = o.state(j), s.state(j)
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(a).max(), 1e-3), j
    lo, lg = o.get(2), s.get(mono.FIELD_LAT)
    assert ((lo > 0) == (lg > 0)).all() and (lo > 0).sum() > 100
    assert np.abs(lo - lg)[lo > 0].max() <= 1e-6


@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_slab_tp06_fp64_parity(torch, layout):
    w = W.slab_ischemic(shape=(23, 19, 11), t_end=25.0)
    w.stimuli = w.stimuli[:1]
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, layout=layout, every=50)
    _assert_f64_levels(w, levels)
    lo, lg = o.get(2), s.get(mono.FIELD_LAT)
    assert ((lo > 0) == (lg > 0)).all() and (lo > 0).sum() > 500


def test_slab_paced_init_fp64_parity(torch):
    """Paced steady-state initial states (normal and ischemic tissue)
    through the same split step."""
    w = W.slab_ischemic(shape=(23, 19, 11), t_end=25.0, init="paced")
    w.stimuli = w.stimuli[:1]
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, every=50)
    _assert_f64_levels(w, levels)
    for j in (1, 2, 3, 5, 8, 12):
        a, b = o.state(j), s.state(j)
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(a).max(), 1e-3), j
    lo, lg = o.get(2), s.get(mono.FIELD_LAT)
    assert ((lo > 0) == (lg > 0)).all() and (lo > 0).sum() > 500


def test_batched_fp64_parity_and_standalone_equality(torch):
    w = W.batched_sheets(n_inst=5, side_lo=20, side_hi=44, t_end=30.0)
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, every=100)
    _assert_f64_levels(w, levels)
    vb = s.get(mono.FIELD_V)
    # each instance equals its own standalone run (bitwise, same precision)
    off = w.mesh.inst_node_off
    for q in (0, 3):
        sl = slice(off[q], off[q + 1])
        sx, sy = w.extra["sides"][q]
        wq = W.batched_sheets(n_inst=5, side_lo=20, side_hi=44, t_end=30.0)
        xyz, conn, _ = W.structured_grid((int(sx), int(sy)), 0.025)
        e0, e1 = w.mesh.inst_elem_off[q], w.mesh.inst_elem_off[q + 1]
        mq = W.Mesh(2, xyz, W.ETYPE_QUAD4, conn, w.mesh.D_elem[e0:e1], w.mesh.sigma[sl])
        sq = mono.Sim(mq, "f64")
        sq.set_cell_model(W.MODEL_TP06, wq.params[:, sl])
        sq.set_lat_threshold(-40.0)
        st = wq.stimuli[0]
        nodes = st.nodes[(st.nodes >= off[q]) & (st.nodes < off[q + 1])] - off[q]
        sq.add_stimulus(nodes, st.t_on, st.duration, st.amplitude)
        # same k decisions as the batched run: replay the oracle's trace slice
        o2 = _oracle(w)
        kt, _ = o2.record_k(w.n_steps)
        o2.step(w.n_steps, w.dt)
        rep = torch.from_numpy(np.ascontiguousarray(kt[:, sl])).cuda()
        sq.ktrace(2, None, rep.data_ptr(), w.n_steps, 0)
        sq.step(w.n_steps, w.dt)
        assert (sq.get(mono.FIELD_V) == vb[sl]).all()


def test_fp32_sheet_error_bounds(torch):
    w = W.sheet_tp06(n=81, t_end=120.0)
    o = _oracle(w)
    s = mono.Sim.from_workload(w, "f32")
    sq = []
    for _ in range(12):
        o.step(100, w.dt)
        s.step(100, w.dt)
        sq.append(np.mean((s.get(mono.FIELD_V) - o.get(0)) ** 2))
    rms = math.sqrt(np.mean(sq))
    lo, lg = o.get(2), s.get(mono.FIELD_LAT)
    assert ((lo > 0) == (lg > 0)).all()
    both = (lo > 0) & (lg > 0)
    assert both.sum() > 1000
    dlat = np.abs(lo - lg)[both].max()
    assert rms <= 0.5 and dlat <= 0.5, (rms, dlat)


# ---------------------------------------------------------------------------
# full-size single launches, sampled against the oracle row by row
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def full_slab():
    w = W.slab_ischemic()                              # 201 x 201 x 51 = 2,060,451 nodes
    return w, _oracle(w)


def _slab_tuned_launch(prec="f32"):
    """The committed tuned launch of the full-size slab in precision prec."""
    import glob
    import json
    import os
    (f,) = glob.glob(os.path.join(os.path.dirname(mono.__file__), "tuned",
                                  f"gfx950_{prec}_stencil13_m2_n2060451_i1_nnz54541351*.json"))
    with open(f) as fh:
        return json.load(fh)["launch"]


@pytest.mark.parametrize("prec,launch", [("f64", "default"), ("f32", "default"),
                                         ("f64", "tuned"), ("f32", "tuned")])
def test_full_slab_single_phases_sampled(torch, full_slab, prec, launch):
    """One diffusion substep and one reaction step of the full 2,060,451-node
    slab, in the default launch shape and in the committed tuned one of each
    precision (the shapes the benchmark times), sampled row by row against
    the oracle."""
    w, o = full_slab
    n = w.mesh.n_nodes
    o.prepare(w.dt)
    y0 = W.random_state(W.MODEL_TP06, n, seed=11)
    rng = np.random.default_rng(12)
    vprev = y0[0] - rng.uniform(-1.5, 1.5, n) * rng.choice([0.0, 0.01, 0.1, 1.0], n)
    s = mono.Sim.from_workload(w, prec)
    if launch == "tuned":
        s.set_launch(**_slab_tuned_launch(prec))
    s.prepare(w.dt)
    rows = np.unique(np.concatenate([rng.integers(0, n, 3000), [0, 1, 200, n - 1, n - 2],
                                     np.arange(n - 300, n)]))
    # one diffusion substep of the second half step at t = 320 ms (S2 is on)
    step = 3200
    for j in range(19):
        s.set(mono.FIELD_STATE0 + j, y0[j])
    s.apply_phase(2, step, 0)
    got = s.get(mono.FIELD_V)[rows]
    ref = o.diffusion_rows(y0[0], step * w.dt + 0.5 * w.dt, 0, rows)
    tol = 1e-12 if prec == "f64" else 2e-5
    assert np.abs(got - ref).max() <= tol * 100
    # one reaction step from the seeded states
    for j in range(19):
        s.set(mono.FIELD_STATE0 + j, y0[j])
    s.set(mono.FIELD_VPREV, vprev)
    s.set(mono.FIELD_LAT, np.full(n, -1.0))
    s.apply_phase(1, 77, 0)
    yr, vpr, lar, kr = o.reaction_nodes(77, rows, y0[:, rows], vprev[rows], np.full(len(rows), -1.0))
    kg = s.get(mono.FIELD_K)[rows]
    if prec == "f64":
        assert (kg == kr).all()
        for j in range(19):
            a, b = yr[j], s.state(j)[rows]
            assert np.abs(a - b).max() <= 1e-10 * max(np.abs(a).max(), 1e-3), j
        assert np.abs(s.get(mono.FIELD_LAT)[rows] - lar).max() <= 1e-9
    else:
        same = kg == kr
        assert same.mean() > 0.995
        assert np.abs(s.state(0)[rows][same] - yr[0][same]).max() <= 0.05


def test_full_slab_graph_equals_eager(torch, full_slab):
    w, _ = full_slab
    a = mono.Sim.from_workload(w, "f32")
    b = mono.Sim.from_workload(w, "f32")
    a.step(64, w.dt)                     # two cached-graph replays
    b.step(64, w.dt, flags=mono.STEP_EAGER)
    assert (a.get(mono.FIELD_V) == b.get(mono.FIELD_V)).all()
    assert (a.state(5) == b.state(5)).all()


def test_graph_remainders_and_capture_only(torch):
    """Step counts that graph_steps does not divide replay a cached remainder
    graph; STEP_CAPTURE captures without running; all equal eager stepping."""
    w = W.slab_ischemic(shape=(27, 21, 9), t_end=20.0)
    a = mono.Sim.from_workload(w, "f32")
    b = mono.Sim.from_workload(w, "f32")
    a.set_launch(graph_steps=16)
    a.step(5, w.dt)
    v0 = a.get(mono.FIELD_V)
    a.step(37, w.dt, flags=mono.STEP_CAPTURE)
    assert a.info()["step"] == 5 and (a.get(mono.FIELD_V) == v0).all()
    for n in (37, 37, 3, 16):
        a.step(n, w.dt)
    b.step(5 + 37 + 37 + 3 + 16, w.dt, flags=mono.STEP_EAGER)
    assert a.info()["step"] == b.info()["step"]
    for f in (mono.FIELD_V, mono.FIELD_LAT, mono.FIELD_K):
        assert (a.get(f) == b.get(f)).all()


@pytest.mark.parametrize("which", ["slab", "batch"])
def test_quiet_chunks_equal_eager(torch, which):
    """Graph chunks in which no stimulus window can open replay a capture
    without the window test; stimuli opening and closing inside chunks, on
    chunk edges and between them give eager stepping's bits."""
    if which == "slab":
        w = W.slab_ischemic(shape=(21, 17, 7), t_end=20.0)
        nodes = w.stimuli[0].nodes
    else:
        w = W.batched_sheets(n_inst=3, side_lo=12, side_hi=24, t_end=20.0)
        nodes = w.stimuli[0].nodes
    amp = w.stimuli[0].amplitude
    # windows: inside the 2nd chunk, starting exactly on a chunk edge
    # (step 16 = 1.6 ms), spanning an edge, and late in the run
    w.stimuli = [W.Stimulus(nodes, 0.25, 0.5, amp), W.Stimulus(nodes, 1.6, 0.3, amp),
                 W.Stimulus(nodes, 3.1, 0.2, amp), W.Stimulus(nodes, 9.55, 1.0, amp)]
    for prec in ("f32", "f64"):
        a = mono.Sim.from_workload(w, prec)
        b = mono.Sim.from_workload(w, prec)
        a.set_launch(graph_steps=8)
        for n in (40, 24, 56):
            a.step(n, w.dt)
        b.step(120, w.dt, flags=mono.STEP_EAGER)
        for f in (mono.FIELD_V, mono.FIELD_LAT, mono.FIELD_K):
            assert (a.get(f) == b.get(f)).all(), (prec, f)
        assert (a.get(mono.FIELD_LAT) >= 0).any()


# ---------------------------------------------------------------------------
# edge cases and failure handling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_nodes", [2, 3, 255, 257, 1000])
def test_ragged_cables(torch, n_nodes):
    w = W.cable_ms(n_nodes=n_nodes, length=0.01 * (n_nodes - 1), t_end=5.0)
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, every=25)
    _assert_f64_levels(w, levels)


@pytest.mark.parametrize("method", [mono.OSTAR, mono.OST])
def test_comparison_methods(torch, method):
    from oracle.oracle import Oracle
    w = W.cable_ms(t_end=10.0)
    dt = 0.01 if method == mono.OST else 0.1
    o = Oracle.from_workload(w, method=method)
    s = mono.Sim.from_workload(w, "f64")
    s.set_method(method)
    n = int(round(10.0 / dt))
    kt, _ = o.record_k(n)
    o.step(n, dt)
    rep = torch.from_numpy(kt).cuda()
    s.ktrace(2, None, rep.data_ptr(), n, 0)
    s.step(n, dt)
    assert s.info()["l"] == 1 and o.info()["l"] == 1
    if method == mono.OST:
        assert s.info()["k_max"] == 1
    vo = o.get(0)
    assert np.abs(s.get(mono.FIELD_V) - vo).max() <= 1e-9 * max(1.0, np.abs(vo).max())


def test_nonfinite_potential_latches(torch):
    w = W.cable_ms(t_end=1.0)
    s = mono.Sim.from_workload(w, "f64")
    V = np.zeros(w.mesh.n_nodes)
    V[50] = np.nan
    s.set(mono.FIELD_V, V)
    s.step(2, w.dt)
    with pytest.raises(mono.MonoError) as e:
        s.sync()
    assert e.value.code == -6
    with pytest.raises(mono.MonoError) as e:
        s.step(1, w.dt)
    assert e.value.code == -4
    s.set(mono.FIELD_V, np.zeros(w.mesh.n_nodes))
    s.step(1, w.dt)
    s.sync()


def test_determinism_two_runs_bitwise(torch):
    w = W.slab_ischemic(shape=(31, 29, 13), t_end=20.0)
    vs = []
    for _ in range(2):
        s = mono.Sim.from_workload(w, "f32")
        s.step(w.n_steps, w.dt)
        vs.append(s.get(mono.FIELD_V))
    assert (vs[0] == vs[1]).all()


# ---------------------------------------------------------------------------
# launch shapes and the autotuner
# ---------------------------------------------------------------------------
def _tuned_launches():
    """The launch shapes committed in the tuning cache (the ones the benchmark
    and the adjoint leg run with)."""
    import glob
    import json
    import os
    d = os.path.join(os.path.dirname(mono.__file__), "tuned")
    out = []
    for f in sorted(glob.glob(os.path.join(d, "*.json"))):
        with open(f) as fh:
            out.append(json.load(fh)["launch"])
    assert out
    return out


@pytest.mark.parametrize("which", ["slab", "batch", "cable"])
def test_launch_shapes_do_not_change_results(torch, which):
    if which == "slab":
        w = W.slab_ischemic(shape=(29, 23, 13), t_end=12.0)
    elif which == "batch":
        w = W.batched_sheets(n_inst=6, side_lo=13, side_hi=37, t_end=12.0)
    else:
        w = W.cable_ms(n_nodes=777, length=7.76, t_end=12.0)
    ref = None
    for cfg in ({}, dict(diff_block=128, diff_rows_per_lane=4, diff_xcd_remap=0, react_block=512,
                         graph_steps=8),
                dict(diff_block=512, diff_rows_per_lane=2, diff_xcd_remap=1, react_block=128,
                     graph_steps=120, react_sort=1),
                dict(react_sort=1, graph_steps=7),
                dict(react_sort=1, react_block=1024, graph_steps=64),
                dict(react_sort=0, react_block=1024, graph_steps=64, diff_classes=0),
                dict(diff_classes=0, diff_rows_per_lane=2, diff_block=128),
                dict(diff_wave_rows=0, diff_rows_per_lane=4, diff_block=512),
                *_tuned_launches()):
        s = mono.Sim.from_workload(w, "f32")
        if cfg:
            s.set_launch(**cfg)
        s.step(w.n_steps, w.dt)
        out = (s.get(mono.FIELD_V), s.state(min(4, s.info()["n_states"] - 1)),
               s.get(mono.FIELD_LAT), s.get(mono.FIELD_K), s.get(mono.FIELD_VPREV))
        if ref is None:
            ref = out
        else:
            for f, (a, b) in enumerate(zip(ref, out)):
                bad = np.flatnonzero(a != b)
                assert bad.size == 0, (cfg, f, bad.size, bad[:5], a[bad[:5]], b[bad[:5]])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("which", ["slab", "sheet", "cable"])
def test_row_classes_match_per_row_arrays(torch, prec, which):
    """Diffusion reading stencil rows by class gives the bits of the per-row
    arrays.  Grid spacings are powers of two so that the node coordinates,
    and with them the element matrices, repeat exactly in FP64 as well."""
    if which == "slab":
        w = W.slab_ischemic(shape=(37, 29, 11), dx=2.0 ** -7, t_end=15.0)
    elif which == "sheet":
        w = W.sheet_tp06(n=61, dx=2.0 ** -5, t_end=15.0)
    else:
        w = W.cable_ms(n_nodes=513, length=4.0, t_end=15.0)
    outs = []
    for cls, rows in ((1, 1), (1, 0), (0, 0)):
        s = mono.Sim.from_workload(w, prec)
        assert s.info()["row_classes"] > 0 and s.info()["grid_rows"] == 1
        s.set_launch(diff_classes=cls, diff_wave_rows=rows)
        s.step(w.n_steps, w.dt)
        outs.append((s.get(mono.FIELD_V), s.get(mono.FIELD_LAT)))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert (a == b).all()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stimulus_windows_on_substep_edges(torch, prec):
    """Stimulus windows that open and close on or between substep start times
    (t = 0.35 falls on a half-step start, 0.4 + 0.1/12 inside a half step,
    an end exactly on a step start, a zero-length window, one opening after
    the run): the single-instance kernels, which test integer substep
    windows, give the bits of the per-row stencil kernel, which tests the
    FP64 start time."""
    w = W.slab_ischemic(shape=(37, 29, 11), dx=2.0 ** -7, t_end=4.0)
    nodes = np.arange(0, w.mesh.n_nodes, 7, dtype=np.int32)
    w.stimuli = [W.Stimulus(nodes, 0.35, 0.3, 40.0),
                 W.Stimulus(nodes[::2], 0.4 + 0.1 / 12.0, 1.2, 30.0),
                 W.Stimulus(nodes[1::3], 1.0, 0.0, 50.0),
                 W.Stimulus(nodes[::5], 2.0, 1e300, 5.0),
                 W.Stimulus(nodes[::4], 3.95, 9.0, 20.0),
                 W.Stimulus(nodes[::3], 50.0, 1.0, 20.0)]
    outs = []
    for cls, rows in ((1, 1), (1, 0), (0, 0)):
        s = mono.Sim.from_workload(w, prec)
        s.set_launch(diff_classes=cls, diff_wave_rows=rows)
        s.step(w.n_steps, w.dt)
        assert s.info()["l"] >= 2
        outs.append((s.get(mono.FIELD_V), s.get(mono.FIELD_LAT)))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert (a == b).all()


def test_row_classes_absent_where_rows_do_not_repeat(torch):
    w = W.batched_sheets(n_inst=3, side_lo=12, side_hi=20)
    assert mono.Sim.from_workload(w, "f32").info()["row_classes"] == 0
    w = W.sheet_tp06(n=41)
    w.mesh.sigma = np.exp(0.2 * np.random.default_rng(0).standard_normal(w.mesh.n_nodes))
    assert mono.Sim.from_workload(w, "f32").info()["row_classes"] == 0


@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_sorted_reaction_fp64_parity(torch, layout):
    """The reaction with the nodes of each workgroup ordered by k, against the
    oracle replaying its k decisions, on the ischemic slab."""
    w = W.slab_ischemic(shape=(25, 21, 9), t_end=25.0)
    _, s, levels, _ = run_pair(torch, w, w.n_steps, "f64", layout, every=40,
                               launch=dict(react_sort=1, graph_steps=16))
    _assert_f64_levels(w, levels)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sorted_reaction_restarts_and_phases(torch, prec):
    """Rewinding the clock, eager steps, single phases and the model-rate
    dV/dt source give the same bits with and without the ordering by k."""
    w = W.slab_ischemic(shape=(23, 19, 9), t_end=20.0)
    outs = []
    for srt in (0, 1):
        s = mono.Sim.from_workload(w, prec)
        s.set_launch(react_sort=srt, graph_steps=5)
        s.step(30, w.dt)
        snap = {f: s.get(f) for f in (mono.FIELD_V, mono.FIELD_VPREV, mono.FIELD_LAT)}
        st = [s.state(j) for j in range(1, s.info()["n_states"])]
        s.step(13, w.dt)
        for f, v in snap.items():
            s.set(f, v)
        for j, v in enumerate(st, start=1):
            s.set(mono.FIELD_STATE0 + j, v)
        s.set_time_level(30)
        s.step(9, w.dt, flags=mono.STEP_EAGER)
        s.step(11, w.dt)
        s.apply_phase(1, 50)
        s.set_method(mono.DAETI, dvdt_source=1)
        s.step(6, w.dt)
        outs.append((s.get(mono.FIELD_V), s.state(3), s.get(mono.FIELD_LAT), s.get(mono.FIELD_K)))
    for a, b in zip(*outs):
        assert (a == b).all()


def test_autotuner_leaves_state_unchanged(torch, tmp_path, monkeypatch):
    from paper_2011_04747_amd import autotune
    monkeypatch.setattr(autotune, "CACHE_DIR", str(tmp_path))
    w = W.slab_ischemic(shape=(41, 37, 15), t_end=10.0)
    a = mono.Sim.from_workload(w, "f32")
    b = mono.Sim.from_workload(w, "f32")
    a.step(30, w.dt)
    b.step(30, w.dt)
    best = autotune.tune(b, w.dt, steps=2, graph_candidates=(8, 16))
    assert b.launch() == best
    assert b.info()["step"] == 30
    a.step(40, w.dt)
    b.step(40, w.dt)
    assert (a.get(mono.FIELD_V) == b.get(mono.FIELD_V)).all()
    again = autotune.tune(b, w.dt)          # cached
    assert again == best


def test_torch_caching_allocator_owns_device_memory(torch):
    """With the allocator hook set to torch's caching allocator the library's
    device buffers come from torch (memory_allocated grows and shrinks with
    the simulation) and results are the same bits; the hook cannot change
    while a simulation exists."""
    w = W.slab_ischemic(shape=(25, 21, 9), t_end=8.0)
    ref = mono.Sim.from_workload(w, "f32")
    ref.step(w.n_steps, w.dt)
    v_ref = ref.get(mono.FIELD_V)
    ref.close()
    import gc
    gc.collect()                      # simulations of earlier tests are destroyed
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    mono.use_torch_allocator()
    try:
        s = mono.Sim.from_workload(w, "f32")
        grown = torch.cuda.memory_allocated() - base
        assert grown >= 20 * w.mesh.n_nodes * 4          # states, potential, operator
        with pytest.raises(mono.MonoError):
            mono.set_allocator()
        s.step(w.n_steps, w.dt)
        assert (s.get(mono.FIELD_V) == v_ref).all()
        s.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        mono.set_allocator()


def test_replayed_k_is_clamped(torch):
    """A replayed trace entry of 0 or above k_max runs (and is recorded) as 1
    or k_max: the run equals one replaying the clamped trace bit for bit."""
    w = W.sheet_tp06(n=23, t_end=3.0)
    n, steps = w.mesh.n_nodes, w.n_steps
    g = np.random.default_rng(11)
    raw = g.integers(1, 11, size=(steps, n)).astype(np.uint8)
    raw[:, ::7] = 0
    raw[:, 3::7] = 200
    kmax = None
    out = []
    for trace in (raw, None):
        s = mono.Sim.from_workload(w, "f64")
        s.prepare(w.dt)
        kmax = s.info()["k_max"]
        if trace is None:
            trace = np.clip(raw, 1, kmax)
        rep = torch.from_numpy(np.ascontiguousarray(trace)).cuda()
        s.ktrace(2, None, rep.data_ptr(), steps, 0)
        s.step(steps, w.dt)
        out.append((s.get(mono.FIELD_V), s.get(mono.FIELD_K),
                    [s.get(mono.FIELD_STATE0 + j) for j in range(1, s.info()["n_states"])]))
        s.close()
    assert kmax == 10
    assert (out[0][1] == np.clip(raw[-1], 1, kmax)).all()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][2], out[1][2]):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# degenerate cases of the method
# ---------------------------------------------------------------------------
def test_daeti_reduces_to_ost_at_the_ost_step(torch):
    """At dt = dt0 the reaction cap k_max = floor(dt/dt0) is 1 and, with
    dt/2 below the stable diffusion step, l = 1: DAETI is then OST, the same
    bits in V, every state and the activation times."""
    w = W.sheet_tp06(n=41, dx=0.05, t_end=8.0)
    out = []
    for method in (mono.DAETI, mono.OST):
        s = mono.Sim.from_workload(w, "f64")
        s.set_method(method)
        s.step(800, 0.01)
        info = s.info()
        assert info["l"] == 1 and info["k_max"] == 1, (method, info["l"], info["k_max"])
        out.append([s.get(mono.FIELD_V), s.get(mono.FIELD_LAT), s.state(4), s.state(9)])
        s.close()
    for a, b in zip(*out):
        assert (a == b).all()


def _single_element(dim):
    """One line, quad or hex element of side 0.01 cm (no row repeats a grid
    pattern wide enough for the row-sharing kernel)."""
    n = 2 ** dim
    xyz = np.array([[(c >> a) & 1 for a in range(dim)] for c in range(n)], float) * 0.01
    order = {1: [0, 1], 2: [0, 1, 3, 2], 3: [0, 1, 3, 2, 4, 5, 7, 6]}[dim]
    conn = np.array([order], np.int32)
    D = np.eye(dim)[None] * 0.001
    return W.Mesh(dim, xyz, n, conn, D)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_single_element_meshes_fp64(torch, dim):
    """The smallest meshes: one element, every node on the boundary and
    stimulated; FP64 against the oracle with its substep counts replayed."""
    m = _single_element(dim)
    p = W.tp06_params(m.n_nodes)
    st = W.Stimulus(np.arange(m.n_nodes, dtype=np.int32), 0.0, 1.0, W.STIM_AMP_TP06_PLANAR)
    w = W.Workload("one_element", m, W.MODEL_TP06, p, [st], 0.1, 30.0, 0.01, "f64", -40.0)
    o, s, levels, nflip = run_pair(torch, w, w.n_steps, every=50)
    _assert_f64_levels(w, levels)
    assert (s.get(mono.FIELD_LAT) > 0).all()


def test_mesh_without_elements_is_rejected(torch):
    """Nodes but no element: no diffusion operator, no stable step (eq. 3
    divides by zero) — rejected at creation."""
    m = W.Mesh(2, np.random.default_rng(0).uniform(0, 1, (5, 2)), 4,
               np.zeros((0, 4), np.int32), np.zeros((0, 2, 2)))
    with pytest.raises(mono.MonoError) as e:
        mono.Sim(m, "f64")
    assert e.value.code == -1
