"""Pins of the oracle's transmural TP06 cell types (heterogeneous tissue,
the widening of Sec. 3's single-cell-type experiments).

The three types differ from the epicardial cell in two conductances and one
gate (ten Tusscher & Panfilov 2006): endocardial cells have G_to = 0.073
instead of 0.294 and an s gate with half-inactivation at -28 mV and a slow
time constant, M cells have G_Ks = 0.098 instead of 0.392.  The pins check
those differences through the rates (closed forms in the epicardial
currents), the gate half-points, and the action potentials they produce: an
endocardial AP without the phase-1 notch and an M-cell AP about 100 ms
longer than the epicardial one.  No GPU.
"""
import numpy as np
import pytest

from paper_2011_04747_amd import workloads as W


def _params(t):
    return W.tp06_types_params(np.array([t]))[:, 0]


def _state(oracle_mod, V):
    y = oracle_mod.model_init(W.MODEL_TP06)
    y[0] = V
    y[13] = 0.6      # r
    y[14] = 0.7      # s
    y[12] = 0.3      # xs
    return y


def test_epicardial_type_is_the_epicardial_model(oracle_mod):
    p6 = np.asarray(W.TP06_PARAM_DEFAULT, float)
    y = oracle_mod.model_init(W.MODEL_TP06)
    y[0] = -20.0
    a = oracle_mod.cell_advance(W.MODEL_TP06, p6, y, 7, 0.1)
    b = oracle_mod.cell_advance(W.MODEL_TP06_TYPES, _params(W.CELL_EPI), y, 7, 0.1)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("V", [-80.0, -30.0, 10.0, 35.0])
def test_conductance_changes_enter_dV_dt_linearly(oracle_mod, V):
    y = _state(oracle_mod, V)
    cur = oracle_mod.tp06_currents(np.asarray(W.TP06_PARAM_DEFAULT, float), y)
    r = {t: oracle_mod.cell_rates(W.MODEL_TP06_TYPES, _params(t), y)[0][0]
         for t in (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)}
    # dV/dt = -I_ion; only I_to (endo) or I_Ks (M) change, by their ratios
    ito_scale = 1.0 - 0.073 / 0.294
    iks_scale = 1.0 - 0.098 / 0.392
    tol = 1e-12 * max(abs(r[W.CELL_EPI]), 1.0)
    assert abs((r[W.CELL_ENDO] - r[W.CELL_EPI]) - ito_scale * cur["Ito"]) <= tol
    assert abs((r[W.CELL_M] - r[W.CELL_EPI]) - iks_scale * cur["IKs"]) <= tol
    assert cur["Ito"] != 0.0 and cur["IKs"] != 0.0


def test_s_gate_half_points_and_endocardial_time_constant(oracle_mod):
    for t, vh in ((W.CELL_EPI, -20.0), (W.CELL_M, -20.0), (W.CELL_ENDO, -28.0)):
        _, inf, _, gate = oracle_mod.cell_rates(W.MODEL_TP06_TYPES, _params(t),
                                                _state(oracle_mod, vh))
        assert gate[14] and abs(inf[14] - 0.5) <= 1e-15
    # endocardial tau_s peaks at V = -67 mV: 1000 + 8 ms
    _, _, tau, _ = oracle_mod.cell_rates(W.MODEL_TP06_TYPES, _params(W.CELL_ENDO),
                                         _state(oracle_mod, -67.0))
    assert abs(tau[14] - 1008.0) <= 1e-12


def _cell_ap(oracle_mod, t):
    """One AP of a two-node cable of cell type t (1 ms stimulus at 1 ms),
    V sampled every 0.1 ms for 600 ms."""
    xyz, conn, et = W.structured_grid((2,), 0.01)
    mesh = W.Mesh(1, xyz, et, conn, np.full((1, 1, 1), 0.001))
    w = W.Workload("cell", mesh, W.MODEL_TP06_TYPES, W.tp06_types_params(np.array([t, t])),
                   [W.Stimulus(np.array([0, 1], np.int32), 1.0, 1.0, 60.0)], 0.1, 600.0,
                   0.01, "f64", -40.0)
    o = oracle_mod.Oracle.from_workload(w)
    V = np.empty((6000, 1))
    for i in range(6000):
        o.step(1, 0.1)
        V[i, 0] = o.get(0)[0]
    apd, _ = oracle_mod.apd90(V, 0.1, -40.0)
    return V[:, 0], apd[0]


def test_transmural_action_potentials(oracle_mod):
    ap = {t: _cell_ap(oracle_mod, t) for t in (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)}
    apd = {t: a for t, (_, a) in ap.items()}
    # the M cell's reduced I_Ks prolongs its AP by roughly 100 ms
    assert 80.0 <= apd[W.CELL_M] - apd[W.CELL_EPI] <= 130.0
    # endocardial and epicardial APs end close together
    assert abs(apd[W.CELL_ENDO] - apd[W.CELL_EPI]) <= 20.0
    # the epicardial phase-1 notch (large I_to) is absent in endocardium:
    # 4 ms after the stimulus ends the endocardial V stays much higher
    i = int(6.0 / 0.1)
    assert ap[W.CELL_ENDO][0][i] >= ap[W.CELL_EPI][0][i] + 8.0
    assert 250.0 <= apd[W.CELL_EPI] <= 330.0


def test_cell_type_row_is_validated(oracle_mod):
    xyz, conn, et = W.structured_grid((3,), 0.01)
    mesh = W.Mesh(1, xyz, et, conn, np.full((2, 1, 1), 0.001))
    p = W.tp06_types_params(np.array([0, 1, 3]))
    w = W.Workload("bad", mesh, W.MODEL_TP06_TYPES, p, [], 0.1, 1.0, 0.01, "f64", -40.0)
    with pytest.raises(Exception):
        oracle_mod.Oracle.from_workload(w)
