"""Paced steady state of the TP06 epicardial cell for the slab workloads.

The paper starts its tissue runs from steady state at a pacing cycle length
of 1000 ms (Sec. 3.1, 3.3).  This script paces one cell of each parameter
set the ischemic slab uses (normal tissue: Ko = 5.4 mM, gNa x 1; ischemic
zone: Ko = 8 mM, gNa x 0.7) with the FP64 CPU oracle and the DAETI step
(dt = 0.1 ms): a two-node cable whose nodes receive the same 1 ms stimulus
of 60 mV/ms every 1000 ms (both nodes stay equal, so no current flows
between them), for BEATS beats.  The state 1000 ms after the last
stimulus (the end of diastole, just before the next beat) is stored with
the largest relative change of any state variable over the last beat.

Writes tp06_paced.json next to this file; workloads.tp06_paced_state()
reads it.  Run:  python tests/golden/pace_tp06.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2011_04747_amd import workloads as W  # noqa: E402

BEATS = 400
CL = 1000.0
DT = 0.1
AMP = 60.0


def pace(ko, gna):
    xyz, conn, et = W.structured_grid((2,), 0.01)
    mesh = W.Mesh(1, xyz, et, conn, np.full((1, 1, 1), 0.001))
    p = W.tp06_params(2)
    p[0] = ko
    p[1] = gna
    stims = [W.Stimulus(np.array([0, 1], np.int32), CL * b, 1.0, AMP) for b in range(BEATS)]
    w = W.Workload("paced_cell", mesh, W.MODEL_TP06, p, stims, DT, CL * BEATS, 0.01, "f64",
                   -40.0)
    o = Oracle.from_workload(w)
    steps = int(round(CL / DT))
    prev = None
    change = None
    apd = None
    for b in range(BEATS):
        o.step(steps, DT)
        y = np.array([o.state(j)[0] for j in range(19)])
        if prev is not None:
            change = float(np.max(np.abs(y - prev) / np.maximum(np.abs(prev), 1e-12)))
        prev = y
    return prev, change


def main():
    out = {"beats": BEATS, "cycle_length_ms": CL, "dt_ms": DT, "stimulus_mV_per_ms": AMP,
           "stimulus_ms": 1.0, "state_order": ["V", "Ki", "Nai", "Cai", "Cass", "CaSR", "Rbar",
                                               "m", "h", "j", "xr1", "xr2", "xs", "r", "s",
                                               "d", "f", "f2", "fCass"]}
    for name, ko, gna in (("normal", 5.4, 1.0), ("ischemic", 8.0, 0.7)):
        t0 = time.time()
        y, ch = pace(ko, gna)
        out[name] = {"Ko": ko, "gNa": gna, "state": y.tolist(), "last_beat_max_rel_change": ch}
        print(name, f"{time.time() - t0:.1f} s", "V", y[0], "Nai", y[2], "change", ch,
              flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tp06_paced.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
