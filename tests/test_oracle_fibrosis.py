"""Pins of the oracle's mixed myocyte/fibroblast tissue (the fibrotic sheet
of Sec. 3.2, with a passive fibroblast membrane standing in for the
MacCannell model).  No GPU.

* A fibroblast node's substep is forward Euler on dV/dt = -g_f (V - E_f):
  after k substeps of h from V0, V = E_f + (V0 - E_f)(1 - g_f h)^k, and its
  other 18 state rows do not move.
* A myocyte node of the mixed model is the epicardial TP06 cell, bit for bit.
* A tissue of fibroblasts only, uniform and unstimulated, follows the
  single-cell closed form at every node through the whole split step
  (diffusion leaves a uniform potential unchanged).
* The fibrotic-sheet workload: the drawn fraction of fibroblasts, and the
  fibroblast conductivity in exactly the elements that hold a fibroblast.
"""
import numpy as np
import pytest

from paper_2011_04747_amd import workloads as W


def _p(cls, g=W.FIBRO_PARAM_DEFAULT[0], E=W.FIBRO_PARAM_DEFAULT[1]):
    return np.concatenate([np.asarray(W.TP06_PARAM_DEFAULT, float), [cls, g, E]])


@pytest.mark.parametrize("k,h", [(1, 0.1), (5, 0.02), (10, 0.01)])
def test_fibroblast_substeps_closed_form(oracle_mod, k, h):
    y = oracle_mod.model_init(W.MODEL_TP06_FIBRO)
    y[0] = 12.5
    g, E = 0.4, -52.0
    out = oracle_mod.cell_advance(W.MODEL_TP06_FIBRO, _p(1, g, E), y, k, k * h)
    want = E + (12.5 - E) * (1.0 - g * h) ** k
    assert out[0] == pytest.approx(want, rel=1e-14, abs=1e-12)
    assert np.array_equal(out[1:], y[1:])


def test_myocyte_node_is_the_epicardial_cell(oracle_mod):
    y = oracle_mod.model_init(W.MODEL_TP06)
    y[0] = -25.0
    a = oracle_mod.cell_advance(W.MODEL_TP06, np.asarray(W.TP06_PARAM_DEFAULT, float), y, 7, 0.1)
    b = oracle_mod.cell_advance(W.MODEL_TP06_FIBRO, _p(0), y, 7, 0.1)
    assert np.array_equal(a, b)
    ra = oracle_mod.cell_rates(W.MODEL_TP06, np.asarray(W.TP06_PARAM_DEFAULT, float), y)
    rb = oracle_mod.cell_rates(W.MODEL_TP06_FIBRO, _p(0), y)
    for u, v in zip(ra, rb):
        assert np.array_equal(u, v)


def test_fibroblast_tissue_follows_the_single_cell(oracle_mod):
    w = W.sheet_fibrotic_tp06(n=13, dx=0.02, fib_frac=1.0, t_end=3.0)
    w.stimuli = []
    n = w.mesh.n_nodes
    y0 = np.repeat(oracle_mod.model_init(W.MODEL_TP06_FIBRO)[:, None], n, axis=1)
    y0[0] = 20.0
    w.init_state = y0
    o = oracle_mod.Oracle.from_workload(w)
    kt, _ = o.record_k(w.n_steps)
    o.step(w.n_steps, w.dt)
    V = o.get(0)
    assert np.all(V == V[0])
    # the same k sequence (uniform tissue) on one cell, outside the mesh
    y = y0[:, 0].copy()
    for s in range(w.n_steps):
        y = oracle_mod.cell_advance(W.MODEL_TP06_FIBRO, _p(1), y, int(kt[s, 0]), w.dt)
    assert V[0] == y[0]
    g, E = W.FIBRO_PARAM_DEFAULT
    # closed form over the recorded substep counts
    v = 20.0
    for s in range(w.n_steps):
        k = int(kt[s, 0])
        v = E + (v - E) * (1.0 - g * w.dt / k) ** k
    assert V[0] == pytest.approx(v, rel=1e-13)


def test_fibrotic_sheet_workload():
    w = W.sheet_fibrotic_tp06(n=41, dx=0.02, fib_frac=0.1, seed=3)
    cls = w.params[6]
    n = w.mesh.n_nodes
    assert int((cls == W.NODE_FIBROBLAST).sum()) == round(0.1 * n)
    assert set(np.unique(cls)) <= {0.0, 1.0}
    has_fib = (cls[w.mesh.conn] == 1.0).any(axis=1)
    dxx = w.mesh.D_elem[:, 0, 0]
    dyy = w.mesh.D_elem[:, 1, 1]
    assert np.allclose(dxx[has_fib], 0.00066) and np.allclose(dxx[~has_fib], 0.002)
    assert np.allclose(dyy, 0.25 * dxx)
    assert np.all(w.mesh.D_elem[:, 0, 1] == 0.0)
    assert w.stimuli[0].t_on == 50.0 and w.stimuli[1].t_on == 200.0


def test_node_class_row_is_checked(oracle_mod):
    w = W.sheet_fibrotic_tp06(n=9, dx=0.02, t_end=1.0)
    w.params[6, 3] = 2.0
    with pytest.raises(RuntimeError):
        oracle_mod.Oracle.from_workload(w)
