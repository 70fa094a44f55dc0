"""Pins of the oracle's TP06 transcription that hold for any correct
transcription and do not retype its rate formulas: where each current
vanishes, which way it flows, the direction of every gate, the L-type
current's removable singularity, and the membrane current as the sum of its
parts.

Each sarcolemmal current of the ten Tusscher-Panfilov model (the cell model of
the paper's Sec. 3) is a conductance times a driving force, so it vanishes at
its ion's equilibrium potential, taken here from the Nernst equation with the
published constants (R 8314.472, T 310 K, F 96485.3415, Na_o 140, Ca_o 2,
K/Na permeability ratio 0.03 for I_Ks), and it is outward (positive) above it.
A current given another ion's reversal potential, a sign error in a driving
force, log10 for ln or a wrong RT/F fails here by many orders of magnitude
more than rounding.  Activation gates rise and inactivation gates fall with
V, between 0 and 1, and every time constant is positive; a sign error in a
steady-state exponent fails here.  These pins together with the charge and
ion balance of the same model leave the numerical constants of the rate
functions (half-activation voltages, slopes, time-constant fits) unpinned."""
import numpy as np
import pytest

from paper_2011_04747_amd import workloads as W

R, T, F = 8314.472, 310.0, 96485.3415
NAO, CAO, PKNA = 140.0, 2.0, 0.03
RTF = R * T / F

V_, KI, NAI, CAI, CASS, CASR, RBAR = 0, 1, 2, 3, 4, 5, 6
M, H, J, XR1, XR2, XS, RG, S, D, FG, F2, FCASS = range(7, 19)
ACTIVATION = {"m": M, "xr1": XR1, "xs": XS, "r": RG, "d": D}
INACTIVATION = {"h": H, "j": J, "xr2": XR2, "s": S, "f": FG, "f2": F2}
SARCOLEMMAL = ("INa", "IK1", "Ito", "IKr", "IKs", "ICaL", "INaCa", "INaK", "IpCa", "IpK",
               "IbNa", "IbCa")


def _state(ki=138.3, nai=7.67, cai=7e-5, cass=7e-5, casr=1.3, gates=0.5):
    from oracle.oracle import model_init
    y = np.array(model_init(W.MODEL_TP06), float)
    y[KI], y[NAI], y[CAI], y[CASS], y[CASR] = ki, nai, cai, cass, casr
    y[7:] = gates
    return y


def _params(ko=5.4):
    p = np.array(W.TP06_PARAM_DEFAULT, float)
    p[0] = ko
    return p


# concentrations well inside and at the edges of what an action potential visits
CONCS = [dict(ki=138.3, nai=7.67, cai=7e-5, ko=5.4),
         dict(ki=120.0, nai=12.0, cai=1e-3, ko=4.0),
         dict(ki=145.0, nai=5.0, cai=2e-5, ko=8.0)]


def _nernst(c):
    ek = RTF * np.log(c["ko"] / c["ki"])
    ena = RTF * np.log(NAO / c["nai"])
    eca = RTF / 2.0 * np.log(CAO / c["cai"])
    eks = RTF * np.log((c["ko"] + PKNA * NAO) / (c["ki"] + PKNA * c["nai"]))
    return {"IK1": ek, "Ito": ek, "IKr": ek, "IpK": ek, "INa": ena, "IbNa": ena, "IbCa": eca,
            "IKs": eks}


@pytest.mark.parametrize("c", CONCS)
def test_each_current_vanishes_at_its_reversal_potential(oracle_mod, c):
    p = _params(c["ko"])
    for name, e in _nernst(c).items():
        y = _state(ki=c["ki"], nai=c["nai"], cai=c["cai"])
        y[V_] = e
        at = oracle_mod.tp06_currents(p, y)[name]
        y[V_] = e + 10.0
        scale = abs(oracle_mod.tp06_currents(p, y)[name])
        assert scale > 0.0, name
        assert abs(at) <= 1e-12 * scale, (name, e, at, scale)


@pytest.mark.parametrize("c", CONCS)
def test_each_current_is_outward_above_its_reversal_potential(oracle_mod, c):
    p = _params(c["ko"])
    for name, e in _nernst(c).items():
        for dv in (-30.0, -3.0, 3.0, 30.0):
            y = _state(ki=c["ki"], nai=c["nai"], cai=c["cai"])
            y[V_] = e + dv
            i = oracle_mod.tp06_currents(p, y)[name]
            assert np.sign(i) == np.sign(dv), (name, dv, i)


@pytest.mark.parametrize("cass", [2e-5, 7e-5, 1e-3])
def test_l_type_current_reversal_and_removable_singularity(oracle_mod, cass):
    """The L-type current is a Goldman-Hodgkin-Katz flux of Ca2+ (z = 2) with
    the model's subspace activity factor 0.25 and its 15 mV shift: it
    vanishes where 0.25 Ca_ss e^(2F(V-15)/RT) = Ca_o, is inward below that
    and continuous through V = 15 mV, where the flux's x/(e^x - 1) factor
    has its removable singularity."""
    p = _params()
    vrev = 15.0 + RTF / 2.0 * np.log(CAO / (0.25 * cass))

    def ical(v):
        y = _state(cass=cass)
        y[V_] = v
        return oracle_mod.tp06_currents(p, y)["ICaL"]

    assert abs(ical(vrev)) <= 1e-12 * abs(ical(vrev - 40.0))
    assert ical(vrev - 5.0) < 0.0 < ical(vrev + 5.0)
    at = ical(15.0)
    for eps in (1e-9, 1e-6, 1e-4):
        for v in (15.0 - eps, 15.0 + eps):
            # Lipschitz: the current changes by a few percent per mV there
            assert abs(ical(v) - at) <= 0.2 * eps * abs(at) + 1e-13 * abs(at), (v, ical(v), at)


def test_membrane_current_is_the_sum_of_the_sarcolemmal_currents(oracle_mod):
    p = _params()
    rng = np.random.default_rng(11)
    for v in (-86.2, -60.0, -20.0, 0.0, 15.0, 30.0):
        y = _state(gates=rng.uniform(0.05, 0.95, 12))
        y[V_] = v
        c = oracle_mod.tp06_currents(p, y)
        total = sum(c[n] for n in SARCOLEMMAL)
        scale = sum(abs(c[n]) for n in SARCOLEMMAL)
        assert abs(c["Iion"] - total) <= 1e-14 * scale
        rate = oracle_mod.cell_rates(W.MODEL_TP06, p, y)[0]
        assert rate[V_] == -c["Iion"]


VS = np.linspace(-100.0, 60.0, 321)


def _gating(oracle_mod, model, kind=None, cass=7e-5):
    p = _params()
    if model == W.MODEL_TP06_TYPES:
        p = np.append(p, kind)
    infs, taus = [], []
    for v in VS:
        y = _state(cass=cass)
        y[V_] = v
        _, inf, tau, gate = oracle_mod.cell_rates(model, p, y)
        assert gate[7:].all() and not gate[:7].any()
        infs.append(inf.copy())
        taus.append(tau.copy())
    return np.array(infs), np.array(taus)


@pytest.mark.parametrize("model,kind", [(W.MODEL_TP06, None),
                                        (W.MODEL_TP06_TYPES, W.CELL_ENDO),
                                        (W.MODEL_TP06_TYPES, W.CELL_M)])
def test_gates_open_and_close_the_right_way(oracle_mod, model, kind):
    inf, tau = _gating(oracle_mod, model, kind)
    g = inf[:, 7:]
    assert (g > 0.0).all() and (g <= 1.0).all()
    assert np.isfinite(tau[:, 7:]).all() and (tau[:, 7:] > 0.0).all()
    for name, i in ACTIVATION.items():
        d = np.diff(inf[:, i])
        assert (d >= 0.0).all() and d.sum() > 0.0, name
        assert inf[0, i] < 0.01 and inf[-1, i] > 0.9, (name, inf[0, i], inf[-1, i])
    for name, i in INACTIVATION.items():
        d = np.diff(inf[:, i])
        assert (d <= 0.0).all() and d.sum() < 0.0, name
        assert inf[0, i] > 0.6, (name, inf[0, i])
    # sodium inactivation: the fast and slow gates share one steady state
    assert np.array_equal(inf[:, H], inf[:, J])
    # the fast inactivation gates of I_Na and I_to and the voltage-dependent
    # L-type inactivation all but close at +60 mV
    for i in (H, J, S, FG):
        assert inf[-1, i] < 0.01, i


def test_calcium_dependent_inactivation_falls_with_subspace_calcium(oracle_mod):
    p = _params()
    vals = []
    for cass in np.geomspace(1e-5, 1e-2, 40):
        y = _state(cass=cass)
        y[V_] = 0.0
        vals.append(oracle_mod.cell_rates(W.MODEL_TP06, p, y)[1][FCASS])
    vals = np.array(vals)
    assert (np.diff(vals) < 0.0).all() and (vals > 0.0).all() and (vals <= 1.0).all()


def test_sr_fluxes_vanish_without_a_gradient(oracle_mod):
    """Release, leak and subspace transfer are driven by concentration
    differences (SR to subspace, SR to cytosol, subspace to cytosol); uptake
    is a pump that rises with cytosolic calcium; release needs open
    ryanodine receptors."""
    p = _params()
    y = _state(cai=3e-4, cass=3e-4, casr=3e-4)
    y[RBAR] = 0.9
    c = oracle_mod.tp06_currents(p, y)
    assert c["Irel"] == 0.0 and c["Ileak"] == 0.0 and c["Ixfer"] == 0.0
    y = _state(cai=1e-4, cass=5e-4, casr=1.3)
    y[RBAR] = 0.0
    c = oracle_mod.tp06_currents(p, y)
    assert c["Irel"] == 0.0 and c["Ileak"] > 0.0 and c["Ixfer"] > 0.0
    ups = []
    for cai in np.geomspace(1e-5, 1e-2, 30):
        ups.append(oracle_mod.tp06_currents(p, _state(cai=cai))["Iup"])
    assert (np.diff(ups) > 0.0).all()


def test_pump_currents_flow_outward_and_saturate(oracle_mod):
    """The Na/K pump moves net positive charge out at every V and speeds up
    with intracellular sodium and extracellular potassium; the sarcolemmal
    calcium pump is outward and rises with cytosolic calcium."""
    for v in (-100.0, -50.0, 0.0, 40.0):
        prev = 0.0
        for nai in (2.0, 5.0, 10.0, 20.0, 40.0):
            y = _state(nai=nai)
            y[V_] = v
            i = oracle_mod.tp06_currents(_params(), y)["INaK"]
            assert i > prev
            prev = i
        prev = 0.0
        for ko in (2.0, 4.0, 5.4, 8.0):
            y = _state()
            y[V_] = v
            i = oracle_mod.tp06_currents(_params(ko), y)["INaK"]
            assert i > prev
            prev = i
    ip = [oracle_mod.tp06_currents(_params(), _state(cai=c))["IpCa"]
          for c in np.geomspace(1e-5, 1e-2, 20)]
    assert ip[0] > 0.0 and (np.diff(ip) > 0.0).all()
