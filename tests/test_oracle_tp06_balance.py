"""A pin of the TP06 cell model's structure that does not retype its rate
formulas: charge and ion balance.

Every TP06 current is carried by one ion species, and the monodomain update
(Sec. 2, step A: forward Euler for V, K_i, Na_i, the buffered calcium totals
and the RyR state; Rush-Larsen for the gates) moves each species by the
current's charge.  So

    Q = K_i + Na_i + 2 (Ca_i,tot + (V_ss / V_c) Ca_ss,tot + (V_sr / V_c) Ca_SR,tot)
        - C_m / (F V_c) V

(buffered totals c + B c / (c + K)) has zero rate, and forward Euler keeps a
linear invariant exactly: every substep must leave Q unchanged up to
rounding, through rest, upstroke, plateau and repolarisation, for every
cell type and for the myocytes of the fibrotic model.  A dropped or wrong
stoichiometric factor (3 I_NaK, 2 I_NaCa), a current given the wrong ion or
sign, a wrong volume ratio or a free concentration stepped instead of a
buffered total each break it by many orders of magnitude more than rounding.
The gate kinetics and current magnitudes are not pinned by it (they stay
parity-unpinned); the balance is checked on the oracle and on the kernel's
own model code built for the host.  Constants: the published TP06 cell
(C_m 0.185 uF, V_c 0.016404, V_sr 0.001094, V_ss 0.00005468, F 96485.3415,
buffers 0.2/0.001, 0.4/0.00025, 10/0.3)."""
import numpy as np
import pytest

from paper_2011_04747_amd import mono
from paper_2011_04747_amd import workloads as W

CM, VC, VSR, VSS, F = 0.185, 0.016404, 0.001094, 0.00005468, 96485.3415
BUF = {3: (0.2, 0.001), 4: (0.4, 0.00025), 5: (10.0, 0.3)}


def _total(c, row):
    B, K = BUF[row]
    return c + B * c / (c + K)


def charge(y):
    ca = _total(y[3], 3) + VSS / VC * _total(y[4], 4) + VSR / VC * _total(y[5], 5)
    return y[1] + y[2] + 2.0 * ca - CM / (F * VC) * y[0]


def _params(model, kind):
    p = np.asarray(W.TP06_PARAM_DEFAULT, float)
    if model == W.MODEL_TP06_TYPES:
        p = np.append(p, kind)
    elif model == W.MODEL_TP06_FIBRO:
        p = np.concatenate([p, [W.NODE_MYOCYTE], W.FIBRO_PARAM_DEFAULT])
    return p


def _run(step, model, kind, n=10000, h=0.05):
    """An action potential from rest (V set to -20 mV, then free running for
    500 ms); returns the largest per-substep change of Q and its drift."""
    from oracle.oracle import model_init
    y = np.array(model_init(model), float)
    y[0] = -20.0
    p = _params(model, kind)
    q0 = charge(y)
    worst, vmax, vmin = 0.0, y[0], y[0]
    for _ in range(n):
        q = charge(y)
        y = step(model, p, y, h)
        worst = max(worst, abs(charge(y) - q))
        vmax, vmin = max(vmax, y[0]), min(vmin, y[0])
    return worst, abs(charge(y) - q0), vmax, vmin, q0


CASES = [(W.MODEL_TP06, None), (W.MODEL_TP06_TYPES, W.CELL_EPI),
         (W.MODEL_TP06_TYPES, W.CELL_ENDO), (W.MODEL_TP06_TYPES, W.CELL_M),
         (W.MODEL_TP06_FIBRO, None)]


@pytest.mark.parametrize("model,kind", CASES)
def test_oracle_tp06_keeps_charge_and_ion_balance(oracle_mod, model, kind):
    worst, drift, vmax, vmin, q0 = _run(
        lambda m, p, y, h: oracle_mod.cell_advance(m, p, y, 1, h), model, kind)
    assert vmax > 0.0 and vmin < -80.0          # an action potential and back to rest
    assert worst <= 1e-12 * abs(q0), worst
    assert drift <= 1e-10 * abs(q0), drift


@pytest.mark.parametrize("model,kind", CASES)
def test_kernel_tp06_code_keeps_charge_and_ion_balance(oracle_mod, model, kind):
    worst, drift, vmax, vmin, q0 = _run(
        lambda m, p, y, h: mono.model_substep_host(m, y, p, h), model, kind)
    assert vmax > 0.0 and vmin < -80.0
    assert worst <= 1e-12 * abs(q0), worst
    assert drift <= 1e-10 * abs(q0), drift


def test_balance_detects_a_wrong_stoichiometry(oracle_mod):
    """The pin is not blind: one substep of the oracle with the Na/K pump's
    sodium counted twice instead of three times (applied here to the
    oracle's own output through its reported I_NaK) breaks Q by the pump's
    charge, far above rounding."""
    from oracle.oracle import model_init
    y = np.array(model_init(W.MODEL_TP06), float)
    p = _params(W.MODEL_TP06, None)
    h = 0.05
    y1 = oracle_mod.cell_advance(W.MODEL_TP06, p, y, 1, h)
    inak = oracle_mod.tp06_currents(p, y)["INaK"]
    assert inak > 0.0
    bad = y1.copy()
    bad[2] += h * inak * CM / (F * VC)           # Na_i moved by 2 I_NaK, not 3
    assert abs(charge(y1) - charge(y)) <= 1e-12 * abs(charge(y))
    assert abs(charge(bad) - charge(y)) > 1e3 * 1e-12 * abs(charge(y))
