"""Launch-shape autotuner for libmono simulations.

Searches, on the simulation it is given and at its current state:
  * diffusion kernel: workgroup size (128/256/512), stencil rows per lane
    (1/2/4; vector loads of the streamed arrays), rows read by class, rows by
    class sharing neighbour rows across lanes (1/2/4 row groups per
    wavefront), and the XCD row remap; on 3D grids that take it, the fused
    half-step kernel (several substeps per launch) and its z planes per
    workgroup;
  * reaction kernel: workgroup size, and whether each workgroup orders its
    nodes by substep count k before advancing them;
  * outer steps per captured HIP graph.
Kernel candidates are timed with the library's per-kernel HIP events
(MONO_STEP_TIMED): diffusion shapes by their time per outer step (fused and
unfused launches do different amounts of work each), reaction shapes per
launch; graph sizes by the wall time of whole steps.  The state is
saved before and restored after, and launch shapes do not change results, so
tuning leaves the simulation exactly as it was.  The choice is cached as JSON
keyed by GPU architecture and problem signature.
"""
from __future__ import annotations

import json
import os
import time
from typing import Optional

import numpy as np

from . import mono

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_DIR = os.environ.get("MONO_TUNE_CACHE", os.path.join(HERE, "tuned"))


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def signature(sim: mono.Sim) -> str:
    i = sim.info()
    lay = "stencil" if i["layout"] == mono.LAYOUT_STENCIL else "ell"
    return (f"{_arch()}_{sim.precision}_{lay}{i['ell_width']}_m{sim.model}_n{sim.n}"
            f"_i{i['n_instances']}_nnz{i['nnz']}" + ("_fz" if i["diff_fused"] else ""))


def _snapshot(sim: mono.Sim):
    S = sim.info()["n_states"]
    fields = [mono.FIELD_VPREV, mono.FIELD_LAT] + [mono.FIELD_STATE0 + j for j in range(S)]
    return sim.info()["step"], {f: sim.get(f) for f in fields}


def _restore(sim: mono.Sim, snap):
    step, fields = snap
    for f, v in fields.items():
        sim.set(f, v)
    sim.set_time_level(step)


def _time_kernels(sim, dt, steps):
    """Diffusion ms per outer step and reaction ms per launch."""
    sim.kernel_times(reset=True)
    sim.step(steps, dt, flags=mono.STEP_TIMED)
    k = sim.kernel_times(reset=True)
    d = k["diffusion_ms"] / steps
    r = k["reaction_ms"] / max(1, k["reaction_launches"])
    return d, r


def tune(sim: mono.Sim, dt: float, steps: int = 8, use_cache: bool = True,
         graph_candidates=(32, 128, 512), verbose: bool = False) -> dict:
    """Pick and apply launch shapes for `sim`; returns the chosen shape."""
    key = signature(sim)
    path = os.path.join(CACHE_DIR, key + ".json")
    if use_cache and os.path.exists(path):
        with open(path) as f:
            best = json.load(f)["launch"]
        sim.set_launch(**best)
        return best
    sim.prepare(dt)
    snap = _snapshot(sim)
    base = sim.launch()
    info = sim.info()
    rpls = (1, 2, 4) if sim.precision == "f32" else (1, 2)
    if info["layout"] != mono.LAYOUT_STENCIL:
        rpls = (1,)
    trials = []
    best_d, best_r = None, None
    _restore(sim, snap)
    _time_kernels(sim, dt, steps)            # warm caches and clocks first
    # per-row arrays (rows per lane 1/2/4), rows by class (1), or rows by
    # class with neighbour rows shared across lanes (row groups 1/2/4)
    shapes = [(0, 0, rpl) for rpl in rpls]
    if info["row_classes"] > 0:
        shapes.append((1, 0, 1))
        if info["grid_rows"]:
            shapes += [(1, 1, g) for g in (1, 2, 4)]
    for blk in (128, 256, 512):
        for cls, rows, rpl in shapes:
            for xcd in (0, 1):
                sim.set_launch(diff_block=blk, diff_rows_per_lane=rpl, diff_xcd_remap=xcd,
                               diff_classes=cls, diff_wave_rows=rows, react_block=blk,
                               react_sort=0, diff_fuse=0)
                _restore(sim, snap)
                d, r = _time_kernels(sim, dt, steps)
                trials.append({"diff_block": blk, "classes": cls, "wave_rows": rows, "rpl": rpl,
                               "xcd": xcd, "diff_ms": d, "react_block": blk, "react_ms": r})
                if verbose:
                    print("tune", trials[-1], flush=True)
                if best_d is None or d < best_d[0]:
                    best_d = (d, blk, rpl, xcd, cls, rows)
                if best_r is None or r < best_r[0]:
                    best_r = (r, blk)
    best = dict(base)
    best.update(diff_block=best_d[1], diff_rows_per_lane=best_d[2], diff_xcd_remap=best_d[3],
                diff_classes=best_d[4], diff_wave_rows=best_d[5], react_block=best_r[1],
                react_sort=0, diff_fuse=0, diff_fuse_planes=0)
    # the fused half step (it reads rows by class); z planes per workgroup,
    # 0 = the library's choice
    if info["diff_fused"] and info["l"] >= 2:
        for planes in (0, 4, 8, 16, 32):
            sim.set_launch(**dict(best, diff_classes=1, diff_fuse=1, diff_fuse_planes=planes))
            _restore(sim, snap)
            d, _ = _time_kernels(sim, dt, steps)
            trials.append({"diff_fuse": 1, "diff_fuse_planes": planes, "diff_ms": d})
            if verbose:
                print("tune", trials[-1], flush=True)
            if d < best_d[0]:
                best_d = (d,) + best_d[1:]
                best.update(diff_classes=1, diff_fuse=1, diff_fuse_planes=planes)
    sort_blocks = (256, 512, 1024) if sim.precision == "f32" else (256, 512)
    for blk in sort_blocks:
        sim.set_launch(**dict(best, react_block=blk, react_sort=1))
        _restore(sim, snap)
        _, r = _time_kernels(sim, dt, steps)
        trials.append({"react_block": blk, "react_sort": 1, "react_ms": r})
        if verbose:
            print("tune", trials[-1], flush=True)
        if r < best_r[0]:
            best_r = (r, blk)
            best.update(react_block=blk, react_sort=1)
    # graph size: wall time of the same steps from the same state (the cost of
    # a step depends on the simulation phase, so every candidate runs the
    # same window)
    gbest = None
    n = max(graph_candidates)
    for g in graph_candidates:
        sim.set_launch(**dict(best, graph_steps=g))
        _restore(sim, snap)
        sim.step(g, dt)          # capture outside the timing
        sim.sync()
        _restore(sim, snap)
        t0 = time.perf_counter()
        sim.step(n, dt)
        sim.sync()
        per = (time.perf_counter() - t0) / n
        trials.append({"graph_steps": g, "ms_per_step": per * 1e3})
        if gbest is None or per < gbest[0]:
            gbest = (per, g)
    best["graph_steps"] = gbest[1]
    sim.set_launch(**best)
    _restore(sim, snap)
    if use_cache:
        os.makedirs(CACHE_DIR, exist_ok=True)
        with open(path, "w") as f:
            json.dump({"key": key, "launch": best, "trials": trials, "dt": dt,
                       "steps_per_trial": steps}, f, indent=1)
    return best
