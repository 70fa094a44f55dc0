"""Heterogeneous tissue on the GPU: TP06 with a transmural cell type per node
(endocardial, M and epicardial layers across a sheet of ventricular wall)
against the FP64 CPU oracle.

Tolerances as in the other parity tests: FP64 with the oracle's k decisions
replayed, 1e-9 of max(|V|, 100 mV) in V and 1e-6 ms in the tracked upstroke
and APD90 times; FP32 free-running, 0.5 ms in those times."""
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


def _oracle_run(w, n_steps, record_k=True):
    from oracle.oracle import Oracle, apd90
    o = Oracle.from_workload(w)
    kt = o.record_k(n_steps)[0] if record_k else None
    buf = o.record_sensors(np.arange(w.mesh.n_nodes, dtype=np.int32), n_steps)
    o.step(n_steps, w.dt)
    apd, tup = apd90(buf, w.dt, w.lat_threshold)
    return o, apd, tup, kt


def _gpu_run(torch, w, n_steps, prec, kt=None, layout=mono.LAYOUT_AUTO):
    s = mono.Sim.from_workload(w, prec, layout=layout)
    if kt is not None:
        rep = torch.from_numpy(kt).cuda()
        rec = torch.zeros_like(rep)
        s.ktrace(3, rec.data_ptr(), rep.data_ptr(), n_steps, 0)
    s.track_apd()
    s.step(n_steps, w.dt)
    torch.cuda.synchronize()
    return s, s.get(mono.FIELD_APD), s.get(mono.FIELD_TUP)


@pytest.mark.parametrize("layout", [mono.LAYOUT_ELL, mono.LAYOUT_STENCIL])
def test_transmural_sheet_fp64_parity(torch, layout):
    w = W.sheet_transmural_tp06(n_wall=61, n_height=17, t_end=500.0)   # 1037 nodes
    n = w.n_steps
    o, apd_o, tup_o, kt = _oracle_run(w, n)
    assert (apd_o > 0).all()
    s, apd_g, tup_g = _gpu_run(torch, w, n, "f64", kt=kt, layout=layout)
    vo, vg = o.get(0), s.get(mono.FIELD_V)
    assert np.abs(vg - vo).max() <= 1e-9 * max(np.abs(vo).max(), 100.0)
    for j in (13, 14, 12):          # r, s, xs: the gates the types change
        a, b = o.state(j), s.state(j)
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(a).max(), 1e-3), j
    assert np.abs(tup_g - tup_o).max() <= 1e-6
    assert np.abs(apd_g - apd_o).max() <= 1e-6


def test_transmural_sheet_fp32_full_size(torch):
    """151 x 51 nodes (1.5 cm of wall): FP32 against the oracle, and the
    layer structure of repolarisation the cell types produce."""
    w = W.sheet_transmural_tp06(t_end=500.0)
    n = w.n_steps
    _, apd_o, tup_o, _ = _oracle_run(w, n, record_k=False)
    _, apd_g, tup_g = _gpu_run(torch, w, n, "f32")
    assert ((apd_g >= 0) == (apd_o >= 0)).all() and (apd_o > 0).all()
    assert np.abs(tup_g - tup_o).max() <= 0.5
    assert np.abs(apd_g - apd_o).max() <= 0.5
    ty = w.params[6]
    mean = {t: apd_g[ty == t].mean() for t in (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)}
    assert mean[W.CELL_M] >= mean[W.CELL_EPI] + 25.0
    assert mean[W.CELL_M] >= mean[W.CELL_ENDO] + 25.0


def test_cell_type_row_is_validated(torch):
    w = W.sheet_transmural_tp06(n_wall=9, n_height=5, t_end=1.0)
    w.params[6, 3] = 3.0
    with pytest.raises(mono.MonoError, match="EINVAL"):
        mono.Sim.from_workload(w, "f64")
    w.params[6, 3] = 0.5
    with pytest.raises(mono.MonoError, match="EINVAL"):
        mono.Sim.from_workload(w, "f64")


def test_cell_type_gradient_entry_is_zero(torch):
    """The type row is a label: mono_backward reports 0 for it while the
    conductance rows get nonzero gradients (the FP64 values against the
    oracle are in test_gpu_adjoint)."""
    w = W.sheet_transmural_tp06(n_wall=21, n_height=7, t_end=8.0)
    sens = np.arange(0, w.mesh.n_nodes, 5, dtype=np.int32)
    target = np.full((w.n_steps, sens.size), -80.0)
    s = mono.Sim.from_workload(w, "f64")
    s.set_sensors(sens, target)
    s.forward_taped(w.n_steps, w.dt, 4)
    _, gp = s.backward()
    torch.cuda.synchronize()
    assert gp.shape == (7,) and gp[6] == 0.0
    assert np.all(gp[1:6] != 0.0)
