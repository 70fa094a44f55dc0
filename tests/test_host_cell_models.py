"""The kernels' cell-model code, evaluated on the host in FP64 (the same
source the reaction kernel compiles), against the oracle's cell models: one
Rush-Larsen / forward-Euler substep (Sec. 2, step A) from seeded states of
every model, including each transmural TP06 cell type.  No GPU."""
import numpy as np
import pytest

from paper_2011_04747_amd import mono
from paper_2011_04747_amd import workloads as W


def _cases(model, rng):
    if model == W.MODEL_MS:
        return [np.asarray(W.MS_PARAM_DEFAULT, float)]
    if model == W.MODEL_LINEAR:
        return [np.array([0.3, -20.0])]
    base = np.asarray(W.TP06_PARAM_DEFAULT, float) * rng.uniform(0.8, 1.2, 6)
    if model == W.MODEL_TP06:
        return [base]
    return [np.append(base, t) for t in (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)]


@pytest.mark.parametrize("model", [W.MODEL_LINEAR, W.MODEL_MS, W.MODEL_TP06,
                                   W.MODEL_TP06_TYPES])
def test_host_substep_matches_oracle(oracle_mod, model):
    rng = np.random.default_rng(11 + model)
    states = W.random_state(model, 40, seed=3 + model).T
    for p in _cases(model, rng):
        for y in states:
            for h in (0.01, 0.1):
                a = oracle_mod.cell_advance(model, p, y, 1, h)
                b = mono.model_substep_host(model, y, p, h)
                scale = np.maximum(np.abs(a), 1e-3)
                assert (np.abs(a - b) <= 1e-11 * scale).all(), (p, y[0], h)


def test_cell_types_differ_where_the_model_says(oracle_mod):
    y = W.random_state(W.MODEL_TP06, 1, seed=5)[:, 0]
    y[0] = 20.0
    p = np.asarray(W.TP06_PARAM_DEFAULT, float)
    out = {t: mono.model_substep_host(W.MODEL_TP06_TYPES, y, np.append(p, t), 0.1)
           for t in (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)}
    epi = mono.model_substep_host(W.MODEL_TP06, y, p, 0.1)
    assert np.array_equal(out[W.CELL_EPI], epi)
    # endocardial: I_to and the s gate change; M: I_Ks changes
    assert out[W.CELL_ENDO][14] != epi[14] and out[W.CELL_M][14] == epi[14]
    assert out[W.CELL_ENDO][0] != epi[0] and out[W.CELL_M][0] != epi[0]
