"""Find the diastolic excitation thresholds of the workloads' stimuli.

The paper stimulates with 1 ms pulses at twice the diastolic threshold
(Sec. 3.1 and Sec. 3.3) without giving the threshold.  This script finds it
by bisection (to 1 % relative) with the FP64 CPU oracle, on small proxies that
keep each stimulus' geometry, spacing, diffusion tensor and cell model:

  ms_cable      1D MS cable, h = 0.01 cm, D = 0.001, x <= 0.05 cm, 2 ms
  tp06_corner   2D TP06 sheet 1 x 1 cm, dx = 0.025, fibres 0->60 deg,
                quarter disc r = 0.25 cm at the corner, 1 ms
  tp06_planar   3D TP06 block 0.4 x 0.04 x 0.5 cm, dx = 0.01, fibres
                rotating -60 -> +60 deg through z, x <= 0.05 cm, 1 ms

A pulse counts as suprathreshold when a node well away from the stimulus
region activates.  Writes stim_thresholds.json next to this file; the
workload constants in paper_2011_04747_amd/workloads.py are twice these.
Run:  python tests/golden/calibrate_stimulus.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2011_04747_amd import workloads as W  # noqa: E402


def fires(w, probe, t_end):
    o = Oracle.from_workload(w)
    o.step(int(round(t_end / w.dt)), w.dt)
    return o.get(2)[probe] > 0.0


def bisect(make, probe, t_end, hi):
    while not fires(make(hi), probe, t_end):
        hi *= 2.0
    lo = 0.0
    while hi - lo > 0.01 * hi:
        mid = 0.5 * (lo + hi)
        if fires(make(mid), probe, t_end):
            hi = mid
        else:
            lo = mid
    return hi


def main():
    out = {"_about": __doc__.strip().splitlines()[0], "method": "bisection, 1% relative, FP64 oracle"}
    # 1D MS cable
    mk = lambda a: W.cable_ms(n_nodes=101, amp=a)
    out["ms_cable"] = bisect(mk, 60, 40.0, 0.1)
    print("ms_cable", out["ms_cable"], flush=True)
    # 2D TP06 corner
    mk = lambda a: W.sheet_tp06(n=41, amp=a)
    w = mk(1.0)
    probe = int(np.argmin(np.sum((w.mesh.xyz - 0.6) ** 2, axis=1)))
    out["tp06_corner"] = bisect(mk, probe, 30.0, 20.0)
    print("tp06_corner", out["tp06_corner"], flush=True)
    # 3D TP06 planar face
    def mk3(a):
        wl = W.slab_ischemic(shape=(41, 5, 51), amp=a, t_end=30.0)
        wl.stimuli = wl.stimuli[:1]
        wl.params = W.tp06_params(wl.mesh.n_nodes)    # healthy tissue
        return wl
    w = mk3(1.0)
    x = w.mesh.xyz
    probe = int(np.argmin((x[:, 0] - 0.3) ** 2 + (x[:, 1] - 0.02) ** 2 + (x[:, 2] - 0.25) ** 2))
    out["tp06_planar"] = bisect(mk3, probe, 30.0, 20.0)
    print("tp06_planar", out["tp06_planar"], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stim_thresholds.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
