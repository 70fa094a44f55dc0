"""The stored paced TP06 states (tests/golden/tp06_paced.json, written by
pace_tp06.py with the oracle) against what physiology fixes: a resting
potential just above the K+ Nernst potential of each tissue's [K+]o (I_K1
dominates at rest), gates at their resting values, and a beat-to-beat drift
small enough to call the cells paced to steady state.  No GPU."""
import json
import math
import os

import numpy as np

from paper_2011_04747_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tp06_paced.json")
RTF = 8314.472 * 310.0 / 96485.3415      # mV


def test_paced_states_rest_near_nernst_and_settled():
    with open(GOLD) as f:
        d = json.load(f)
    assert d["beats"] >= 200 and d["cycle_length_ms"] == 1000.0
    ps = W.tp06_paced_state()
    for name in ("normal", "ischemic"):
        y = ps[name]
        ko = d[name]["Ko"]
        ek = RTF * math.log(ko / y[1])
        # at rest V sits within a few mV above E_K
        assert 0.0 < y[0] - ek < 3.0, (name, y[0], ek)
        # m ~ 0, h and j open, fCass ~ 1, concentrations physiological
        assert y[7] < 0.05 and y[8] > 0.3 and y[9] > 0.3
        assert 120.0 < y[1] < 145.0 and 5.0 < y[2] < 15.0 and 0.0 < y[3] < 2e-4
        assert d[name]["last_beat_max_rel_change"] < 2e-3
    # hyperkalaemia depolarises the ischemic zone's resting potential
    assert ps["ischemic"][0] > ps["normal"][0] + 5.0


def test_paced_slab_initial_state_by_zone():
    w = W.slab_ischemic(shape=(21, 17, 11), init="paced")
    ps = W.tp06_paced_state()
    isc = w.params[0] == 8.0
    assert isc.any() and (~isc).any()
    assert np.array_equal(w.init_state[:, isc], np.repeat(ps["ischemic"][:, None], isc.sum(), 1))
    assert np.array_equal(w.init_state[:, ~isc],
                          np.repeat(ps["normal"][:, None], (~isc).sum(), 1))
