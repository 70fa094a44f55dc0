"""Throughput benchmark of the DAETI monodomain solver on one MI355X.

Workload: the 3D TP06 slab, 2 x 2 x 0.5 cm at dx = 0.01 cm (201 x 201 x 51 =
2,060,451 nodes), trilinear hexes, fibres rotating -60..+60 deg through the
wall, a seeded ischemic ellipsoid ([K+]o = 8 mM, g_Na x 0.7), S1 at x = 0 and
a cross-field S2 at 320 ms, dt = 0.1 ms, FP32 state and operator with FP64
time, stable-step estimate and activation times.

A step is one outer DAETI step (B(dt/2) A(dt) B(dt/2)) over the whole mesh;
`value` is node-updates per second over the K timed steps (inputs resident in
HBM), timed with events on the simulation's stream between device-wide
synchronisations.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("node-updates/s (ionic+diffusion) at stated accuracy vs FP64 plain; "
          "adjoint/fwd ratio")
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# the same FP32 vector units without packed (two-wide) instructions, which
# the build disables: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PLAIN_VALU_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6


def _sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel, workload, launch):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (copy-calibrated), or None when absent, taken on another workload
    or launch shape, or when the kernel's sources have changed since."""
    if workload is None:
        return None
    suffix = "" if workload == "slab" else f"_{workload}"
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}{suffix}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    keys = {"diffusion": ("diff_block", "diff_rows_per_lane", "diff_xcd_remap", "diff_classes",
                          "diff_wave_rows", "diff_fuse", "diff_fuse_planes"),
            "reaction": ("react_block", "react_sort")}[kernel]
    tl = t.get("launch") or {}
    if t.get("bench_workload") != workload or any(tl.get(k) != launch.get(k) for k in keys):
        return None
    if _sha(t["sources"]) != t["source_sha"]:
        return None
    return t["bytes_per_launch"]


LEVEL_EVERY = 1000     # outer steps between compared levels of the whole run (100 ms)


def full_run(w, stream, launch, layout, with_accuracy):
    """The workload's whole simulated interval from t = 0 (every phase: the
    S1 front crossing resting tissue, plateau, repolarisation, S2 and
    re-entry), graph-replayed and timed with HIP events on the simulation's
    stream; then the same run again with the substep statistics on for the
    mean k and the wavefront efficiency of the reaction, stopping every
    100 ms to read the potential; and (with_accuracy) the same levels from
    the FP64 path for the accuracy of the FP32 run over the whole interval."""
    import torch
    from paper_2011_04747_amd import mono
    steps = w.n_steps
    sim = mono.Sim.from_workload(w, "f32", stream=stream.cuda_stream, layout=layout)
    sim.set_launch(**launch)
    sim.step(steps, w.dt, flags=mono.STEP_CAPTURE)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(steps, w.dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    lat = sim.get(mono.FIELD_LAT)
    sim.close()
    marks = list(range(LEVEL_EVERY, steps + 1, LEVEL_EVERY))
    if not marks or marks[-1] != steps:
        marks.append(steps)

    def levels(prec, stats):
        sm = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream, layout=layout)
        if prec == "f32":
            sm.set_launch(**launch)
        if stats:
            sm.stats_enable(True)
        out, done = [], 0
        for m in marks:
            sm.step(m - done, w.dt)
            done = m
            out.append(sm.get(mono.FIELD_V))
        st = sm.stats() if stats else None
        lt = sm.get(mono.FIELD_LAT)
        sm.close()
        return out, lt, st

    v32, lat32, (ksum, kwave, node_steps, ksat) = levels("f32", True)
    res = {"level_run_equals_timed_run": bool(np.array_equal(lat32, lat)), "steps": steps, "simulated_ms": steps * w.dt, "ms": ms,
           "node_updates_per_s": w.mesh.n_nodes * steps / (ms * 1e-3),
           "mean_k": ksum / max(1, node_steps), "wave_efficiency": ksum / max(1, kwave),
           "k_at_kmax_frac": ksat / max(1, node_steps),
           "activated_frac": float((lat >= 0).mean())}
    if with_accuracy:
        v64, lat64, _ = levels("f64", False)
        rms = [float(np.sqrt(np.mean((a - b) ** 2))) for a, b in zip(v32, v64)]
        pre = [r for m, r in zip(marks, rms) if m * w.dt <= 300.0 + 1e-9]
        both = (lat32 >= 0) & (lat64 >= 0)
        res["accuracy"] = {
            "reference": "FP64 path of the same kernels over the same run (FP64 parity with the "
                         "oracle is tested on this slab's geometry at dx 0.05 cm over 0-350 ms)",
            "levels_ms": [m * w.dt for m in marks],
            "v_rms_mV_per_level": rms,
            "v_rms_mV_0_300ms": float(np.sqrt(np.mean(np.square(pre)))) if pre else None,
            "v_rms_mV_whole_run": float(np.sqrt(np.mean(np.square(rms)))),
            "v_max_mV_whole_run": float(max(np.abs(a - b).max() for a, b in zip(v32, v64))),
            "lat_max_ms": float(np.abs(lat32 - lat64)[both].max()) if both.any() else None,
            "activated_equal": bool(((lat32 >= 0) == (lat64 >= 0)).all())}
    return res


def time_window(w, prec, stream, steps, warmup, repeats, layout, tune):
    """K outer steps after W warm-up steps of workload w in precision prec,
    graph-replayed and timed with events on the simulation's stream `repeats`
    times from the same state (median); then the same window once more with
    the substep statistics on (mean k), and the diffusion substep timed in a
    graph of back-to-back substeps."""
    import torch
    from paper_2011_04747_amd import mono
    sim = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream, layout=layout)
    sim.step(warmup, w.dt)
    launch = sim.launch()
    if tune:
        from paper_2011_04747_amd import autotune
        launch = autotune.tune(sim, w.dt)
    sim.step(steps, w.dt, flags=mono.STEP_CAPTURE)
    info = sim.info()
    fields = [mono.FIELD_VPREV, mono.FIELD_LAT] + \
        [mono.FIELD_STATE0 + j for j in range(info["n_states"])]
    snap = (info["step"], {f: sim.get(f) for f in fields})

    def restore():
        for f, v in snap[1].items():
            sim.set(f, v)
        sim.set_time_level(snap[0])

    times = []
    for r in range(max(1, repeats)):
        if r:
            restore()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(steps, w.dt)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    ms = sorted(times)[len(times) // 2]
    restore()
    sim.stats_enable(True)
    sim.step(steps, w.dt)
    ksum, _, node_steps, _ = sim.stats()
    sim.stats_enable(False)
    L = max(sim.info(q)["l"] for q in range(info["n_instances"]))
    d_us = 1e3 * sim.time_diffusion(64 * 2 * L)
    sim.close()
    n = w.mesh.n_nodes
    return {"ms": ms, "repeats_ms": times, "node_updates_per_s": n * steps / (ms * 1e-3),
            "ms_per_step": ms / steps, "mean_k": ksum / max(1, node_steps),
            "substeps_per_step": ksum / steps, "diffusion_us": d_us, "L": L,
            "reaction_us": 1e3 * ms / steps - 2 * L * d_us, "info": info, "launch": launch}


def _diff_row_bytes(info, launch, es):
    """Algorithmic HBM bytes per row of one diffusion substep (value size es)."""
    from paper_2011_04747_amd import mono
    P = info["ell_width"]
    by_class = (info["layout"] == mono.LAYOUT_STENCIL and info["row_classes"] > 0
                and launch.get("diff_classes", 1))
    if by_class:
        b = 2 * es + 2                 # V in, V out, class id
    elif info["layout"] == mono.LAYOUT_STENCIL:
        b = (P + 3) * es               # own edges, 1/m, V in, V out
    else:
        b = P * (es + 4) + 2 * es      # (value, column) per slot, V in, V out
    if info["n_instances"] > 1:
        b += 4                         # instance id of the row
    return b


def _react_node_bytes(w, info, es):
    """Algorithmic HBM bytes per node of one reaction launch (value size es):
    the S states (V among them), V_prev and the per-node parameter rows read;
    the S states, V_prev and the 1-byte k written.  Parameter rows that are
    uniform over the mesh travel as kernel arguments, and the FP64 activation
    time is read and written only where V crosses the threshold in that
    step, so neither is counted."""
    import numpy as np
    p = np.asarray(w.params) if w.params is not None else np.zeros((0, 1))
    pernode = sum(1 for r in range(p.shape[0]) if (p[r] != p[r][0]).any())
    S = info["n_states"]
    return (S + 1 + pernode) * es + (S + 1) * es + 1


def _model_ops():
    """Operation count of one TP06 substep at the library's initial state."""
    from paper_2011_04747_amd import mono
    from paper_2011_04747_amd import workloads as W
    tiny = mono.Sim.from_workload(W.sheet_tp06(n=2, t_end=0.1), "f64")
    rest = [float(tiny.get(mono.FIELD_STATE0 + j)[0]) for j in range(tiny.info()["n_states"])]
    tiny.close()
    ops = mono.model_flops(W.MODEL_TP06, rest, W.TP06_PARAM_DEFAULT)
    return ops, ops["add"] + ops["mul"] + ops["div"] + ops["exp"] + ops["log"] + ops["sqrt"]


def one_graph_run(w, prec, stream, launch, layout):
    """The workload's whole interval from t = 0 captured as one HIP graph and
    replayed by one launch (capture outside the timing), timed with events on
    the simulation's stream."""
    import torch
    from paper_2011_04747_amd import mono
    n = w.n_steps
    sim = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream, layout=layout)
    sim.set_launch(**dict(launch, graph_steps=min(n, 8192)))
    t0 = time.perf_counter()
    sim.step(n, w.dt, flags=mono.STEP_CAPTURE)
    sim.sync()
    capture_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(n, w.dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    sim.close()
    return {"steps": n, "simulated_ms": n * w.dt, "graph_launches": (n + 8191) // 8192,
            "ms": ms, "node_updates_per_s": w.mesh.n_nodes * n / (ms * 1e-3),
            "capture_s": capture_s}


def other_leg(kind, w, prec, stream, args, layout, name):
    """Throughput of another workload (or precision) over the same window,
    with the roofline of its diffusion and reaction kernels."""
    r = time_window(w, prec, stream, args.steps, args.warmup, 3, layout, not args.no_tune)
    info, launch = r["info"], r["launch"]
    es = 8 if prec == "f64" else 4
    row_b = _diff_row_bytes(info, launch, es)
    _, f_model = _model_ops()
    flops = r["substeps_per_step"] * f_model
    peak = FP64_VECTOR_PEAK_TFLOPS if prec == "f64" else FP32_VECTOR_PEAK_TFLOPS
    # committed HBM traffic of this workload and launch shape (FP32 counters)
    tkey = kind if kind in ("batched", "tets") and prec == "f32" else None
    out = {"workload": name, "dtype": prec, "nodes": w.mesh.n_nodes, "steps": args.steps,
           "warmup": args.warmup, "value": r["node_updates_per_s"], "unit": "node-updates/s",
           "ms_per_step": r["ms_per_step"], "repeats_ms": r["repeats_ms"], "launch": launch,
           "l": r["L"], "mean_k": r["mean_k"],
           "diffusion": {"avg_us": r["diffusion_us"], "bytes_per_row": row_b,
                         "traffic": _traffic("diffusion", tkey, launch),
                         "launches_per_half_step": info["diff_launches"] or r["L"],
                         "achieved_GBs": w.mesh.n_nodes * row_b / (r["diffusion_us"] * 1e-6) / 1e9,
                         "frac_hbm": w.mesh.n_nodes * row_b / (r["diffusion_us"] * 1e-6) / 1e9
                         / HBM_PEAK_GBS,
                         "ms_per_step": 2 * r["L"] * r["diffusion_us"] * 1e-3},
           "reaction": {"avg_us": r["reaction_us"],
                        "traffic": _traffic("reaction", tkey, launch),
                        "bytes_per_node": _react_node_bytes(w, info, es),
                        "frac_hbm": w.mesh.n_nodes * _react_node_bytes(w, info, es)
                        / (r["reaction_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                        "achieved_TFLOPs": flops / (r["reaction_us"] * 1e-6) / 1e12,
                        "peak_TFLOPs": peak,
                        "frac": flops / (r["reaction_us"] * 1e-6) / 1e12 / peak}}
    return out


def _host_cpu():
    """CPU model, physical cores and logical CPUs of this host (lscpu)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    def num(k):
        try:
            return int(info.get(k, ""))
        except ValueError:
            return None
    cores = (num("Core(s) per socket") or 0) * (num("Socket(s)") or 0) or None
    return {"cpu_model": info.get("Model name"), "physical_cores": cores,
            "logical_cpus": num("CPU(s)"), "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(w, steps, steps_1t):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the workload:
    `steps` outer steps on all threads, then `steps_1t` more on one thread.
    The oracle is compiled -O3 -march=native for this host first."""
    from oracle import build as oracle_build
    from oracle import oracle as oracle_mod
    oracle_mod.use_library(oracle_build.build_native())
    from oracle.oracle import Oracle, get_threads, set_threads
    o = Oracle.from_workload(w)
    o.prepare(w.dt)
    threads = get_threads()
    t0 = time.perf_counter()
    o.step(steps, w.dt)
    el = time.perf_counter() - t0
    out = {"value": w.mesh.n_nodes * steps / el, "unit": "node-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"full {w.mesh.n_nodes}-node slab, FP64, first {steps} outer steps "
                     f"from t=0 (assembly excluded), {el:.1f} s, {threads} OpenMP threads",
           "build": "g++ -O3 -march=native -ffp-contract=off -fopenmp", "host": _host_cpu()}
    if steps_1t > 0:
        set_threads(1)
        t0 = time.perf_counter()
        o.step(steps_1t, w.dt)
        el1 = time.perf_counter() - t0
        set_threads(threads)
        out["value_1_thread"] = w.mesh.n_nodes * steps_1t / el1
        out["sample_1_thread"] = f"the next {steps_1t} outer steps on 1 thread, {el1:.1f} s"
    return out


def adjoint_leg(stream, with_accuracy, tune=True):
    """Adjoint/forward wall-time ratio on the 3D adjoint slab (101x101x26,
    512 sensors, loss over 300 ms, checkpoints every 50 steps, FP32)."""
    import torch
    from paper_2011_04747_amd import mono
    from paper_2011_04747_amd import workloads as W
    w = W.adjoint_slab(precision="f32")
    n_steps = w.n_steps
    ns = len(w.sensors)
    ck = w.extra["ckpt_every"]
    # synthetic measurements: the same tissue with the perturbed conductivity
    mt = W.Mesh(w.mesh.dim, w.mesh.xyz, w.mesh.etype, w.mesh.conn, w.mesh.D_elem,
                w.extra["sigma_target"])
    wt = W.Workload(w.name, mt, w.model, w.params, w.stimuli, w.dt, w.t_end, w.dt0, "f32",
                    w.lat_threshold)
    st = mono.Sim.from_workload(wt, "f32", stream=stream.cuda_stream)
    st.set_sensors(w.sensors, np.zeros((0, ns)))
    target = st.sample_sensors(n_steps, w.dt, ns)
    st.close()

    # launch shape of the FP32 runs: tuned (or read from the tuning cache)
    # after 64 steps of the forward run
    launch = None
    if tune:
        from paper_2011_04747_amd import autotune
        s = mono.Sim.from_workload(w, "f32", stream=stream.cuda_stream)
        s.step(64, w.dt)
        launch = autotune.tune(s, w.dt)
        s.close()

    def run(prec, taped, ktrace=None, sched=("uniform", 0), round_init=False):
        s = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream)
        if launch and prec == "f32":
            s.set_launch(**launch)
        s.set_sensors(w.sensors, target)
        if round_init:
            # the FP32 run's initial state (every value rounded to FP32), in FP64
            for j in range(s.info()["n_states"]):
                s.set(mono.FIELD_STATE0 + j,
                      s.get(mono.FIELD_STATE0 + j).astype(np.float32).astype(np.float64))
        if ktrace is not None:
            mode, buf = ktrace
            if mode == 1:
                s.ktrace(1, buf.data_ptr(), None, n_steps, 0)
            else:
                s.ktrace(2, None, buf.data_ptr(), n_steps, 0)
        s.set_checkpointing(*sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if not taped:
            s.step(n_steps, w.dt)
            s.sync()
            out = (time.perf_counter() - t0, None)
        else:
            loss = s.forward_taped(n_steps, w.dt, ck)
            t1 = time.perf_counter()
            gs, gp = s.backward()
            t2 = time.perf_counter()
            out = (t1 - t0, t2 - t1, loss, gs, gp, s.checkpoint_info())
        s.close()
        return out

    run("f32", False)                      # warm-up (graph capture, code load)
    t_fwd = run("f32", False)[0]
    t_tf, t_bw, loss, gs, gp, ci = run("f32", True)
    names = ("gNa", "gCaL", "gKr", "gKs", "gK1")
    res = {"workload": f"adjoint_tp06_3d 101x101x26 ({w.mesh.n_nodes} nodes), {ns} sensors, "
                       f"{n_steps} steps, checkpoint every {ck}, FP32",
           "launch": launch, "forward_s": t_fwd, "taped_forward_s": t_tf, "backward_s": t_bw,
           "adjoint_over_forward": (t_tf + t_bw) / t_fwd, "loss": loss,
           "grad_sigma_l2": float(np.linalg.norm(gs)),
           "grad_scalings": {k: float(gp[i]) for i, k in enumerate(names, start=1)},
           "checkpointing": {"uniform": {"snapshots": ci["snapshots"],
                                         "snapshot_MB": ci["snapshot_bytes"] / 1e6,
                                         "tape_MB": ci["tape_bytes"] / 1e6,
                                         "segment_advances": ci["advances"]}}}
    # binomial checkpointing in a few snapshot buffers: same gradients,
    # less memory, forward advances in the reverse sweep
    for slots in (8, 3):
        tb_tf, tb_bw, lb, gsb, gpb, cib = run("f32", True, sched=("binomial", slots))
        res["checkpointing"][f"binomial_{slots}"] = {
            "snapshots": cib["snapshots"], "snapshot_MB": cib["snapshot_bytes"] / 1e6,
            "tape_MB": cib["tape_bytes"] / 1e6, "segment_advances": cib["advances"],
            "taped_forward_s": tb_tf, "backward_s": tb_bw,
            "adjoint_over_forward": (tb_tf + tb_bw) / t_fwd,
            "gradients_equal_uniform": bool(lb == loss and np.array_equal(gsb, gs)
                                            and np.array_equal(gpb, gp))}
    if with_accuracy:
        # same k decisions in both precisions: record the FP32 run's, replay in FP64
        kt = torch.zeros((n_steps, w.mesh.n_nodes), dtype=torch.uint8, device="cuda")
        _, _, loss, gs, gp, _ = run("f32", True, (1, kt))
        _, _, loss64, gs64, gp64, _ = run("f64", True, (2, kt))
        # conditioning: the FP64 adjoint from the FP32-rounded initial state
        _, _, loss64r, gs64r, gp64r, _ = run("f64", True, (2, kt), round_init=True)
        del kt

        def rel(a, b):
            return {k: float(abs(a[i] - b[i]) / abs(b[i])) for i, k in enumerate(names, start=1)}
        res["fp32_vs_fp64"] = {
            "note": "FP64 adjoint of the same kernels replaying the FP32 run's k decisions",
            "grad_sigma_cosine": float(np.dot(gs, gs64) / (np.linalg.norm(gs) * np.linalg.norm(gs64))),
            "grad_sigma_rel_l2": float(np.linalg.norm(gs - gs64) / np.linalg.norm(gs64)),
            "grad_scalings_max_rel": float(np.max(np.abs(gp[1:] - gp64[1:]) / np.abs(gp64[1:]).max())),
            "grad_scalings_rel": rel(gp, gp64),
            "grad_scalings_cosine": float(np.dot(gp[1:], gp64[1:]) /
                                          (np.linalg.norm(gp[1:]) * np.linalg.norm(gp64[1:]))),
            "loss_rel": float(abs(loss - loss64) / loss64)}
        # a loss whose residuals all have one sign (target = the FP64 run's own
        # potentials minus 5 mV): no cancellation between sensors and times
        st = mono.Sim.from_workload(w, "f64", stream=stream.cuda_stream)
        st.set_sensors(w.sensors, np.zeros((0, ns)))
        own = st.sample_sensors(n_steps, w.dt, ns)
        st.close()
        kt = torch.zeros((n_steps, w.mesh.n_nodes), dtype=torch.uint8, device="cuda")
        saved = target
        target = own - 5.0
        _, _, lo32, gso32, gpo32, _ = run("f32", True, (1, kt))
        _, _, lo64, gso64, gpo64, _ = run("f64", True, (2, kt))
        target = saved
        del kt
        res["fp32_vs_fp64_one_sign_residuals"] = {
            "note": "target = FP64 potentials at the sensors minus 5 mV, same k decisions; the "
                    "scaling gradients of the perturbed-conductivity loss are small remainders "
                    "of sums whose terms change sign (compare their magnitudes with these)",
            "grad_scalings_rel": rel(gpo32, gpo64),
            "grad_scalings": {k: float(gpo64[i]) for i, k in enumerate(names, start=1)},
            "grad_sigma_rel_l2": float(np.linalg.norm(gso32 - gso64) / np.linalg.norm(gso64)),
            "loss_rel": float(abs(lo32 - lo64) / lo64)}
        res["fp64_conditioning"] = {
            "note": "FP64 adjoint from the initial state rounded to FP32 against FP64 from the "
                    "exact one (same k decisions): the change an FP32-sized perturbation of the "
                    "input alone makes",
            "grad_scalings_max_rel": float(np.max(np.abs(gp64r[1:] - gp64[1:]) /
                                                  np.abs(gp64[1:]).max())),
            "grad_scalings_rel": rel(gp64r, gp64),
            "grad_sigma_rel_l2": float(np.linalg.norm(gs64r - gs64) / np.linalg.norm(gs64)),
            "loss_rel": float(abs(loss64r - loss64) / loss64)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=320)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--layout", default="auto", choices=["auto", "ell", "stencil"])
    ap.add_argument("--workload", default="slab", choices=["slab", "batched", "tets"])
    ap.add_argument("--init", default="rest", choices=["rest", "paced"],
                    help="initial state of the slab: published values or paced steady state")
    ap.add_argument("--order", default="rcm", choices=["rcm", "morton", "random", "grid"],
                    help="node order of the tetrahedral slab")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--cpu-steps-1t", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip timing the workload's whole simulated interval")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the FP64, batched and tetrahedral windows")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"],
                    help="arithmetic of the timed window (f64: FP64 state and operator)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo decomposition is a design, not a build).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2011_04747_amd import mono
    from paper_2011_04747_amd import workloads as W

    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    layout = {"auto": mono.LAYOUT_AUTO, "ell": mono.LAYOUT_ELL,
              "stencil": mono.LAYOUT_STENCIL}[args.layout]
    if args.workload == "slab":
        w = W.slab_ischemic(precision="f32", init=args.init)
        wl_name = ("slab_tp06_3d_ischemic 201x201x51 (2,060,451 nodes), Q1 hexes, dx=0.01 cm, "
                   "dt=0.1 ms, S1+S2" +
                   (", paced initial state (400 beats at 1000 ms)" if args.init == "paced"
                    else ""))
    elif args.workload == "tets":
        w = W.slab_ischemic_tets(precision="f32", order=args.order)
        order_name = {"rcm": "RCM", "morton": "Morton (Z-order)", "random": "shuffled",
                      "grid": "grid"}[args.order]
        wl_name = ("slab_tp06_3d_ischemic_tets 201x201x51 (2,060,451 nodes, "
                   f"{w.mesh.n_elems:,} linear tetrahedra), {order_name} node order, dx=0.01 cm, "
                   "dt=0.1 ms, S1+S2")
    else:
        w = W.batched_sheets(precision="f32")
        wl_name = (f"batched_tp06_2d: 64 sheets, sides U{{50..400}} seed 4, "
                   f"{w.mesh.n_nodes} nodes, log-normal sigma, dt=0.1 ms")
    # the committed traffic counters of the tetrahedral slab were taken in RCM order
    traffic_key = args.workload if args.workload != "tets" or args.order == "rcm" else None
    n = w.mesh.n_nodes
    stream = torch.cuda.Stream()
    prec = args.precision
    es = 8 if prec == "f64" else 4
    sim = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream, layout=layout)
    launch = sim.launch()
    info = sim.info()

    # warm-up; the launch shape is tuned (or read from the tuning cache) at
    # the state the timed window starts from (tuning restores the state);
    # then the graphs the window replays (graph_steps steps and the remainder
    # of K) are captured outside it
    sim.step(args.warmup, w.dt)
    if not args.no_tune:
        from paper_2011_04747_amd import autotune
        launch = autotune.tune(sim, w.dt)
    sim.step(args.steps, w.dt, flags=mono.STEP_CAPTURE)
    # the window is timed `repeats` times from the same state (restored from a
    # snapshot); value = the median
    snap = None
    if args.repeats > 1:
        fields = [mono.FIELD_VPREV, mono.FIELD_LAT] + \
            [mono.FIELD_STATE0 + j for j in range(info["n_states"])]
        snap = (sim.info()["step"], {f: sim.get(f) for f in fields})
    times = []
    for r in range(max(1, args.repeats)):
        if snap and r:
            for f, v in snap[1].items():
                sim.set(f, v)
            sim.set_time_level(snap[0])
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        t0 = time.perf_counter()
        sim.step(args.steps, w.dt)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append((ev0.elapsed_time(ev1), time.perf_counter() - t0))
    ms, wall = sorted(times)[len(times) // 2]
    info = sim.info()
    value = n * args.steps / (ms * 1e-3)

    v32 = sim.get(mono.FIELD_V)
    l32 = sim.get(mono.FIELD_LAT)
    sim.close()

    # per-kernel durations over the same simulated window: an identical
    # simulation repeats the warm-up, then runs the K timed steps one launch at
    # a time, each kernel bracketed by HIP events on the simulation's stream;
    # the substep counts k each node took are read back between steps
    sim = mono.Sim.from_workload(w, prec, stream=stream.cuda_stream, layout=layout)
    sim.set_launch(**launch)
    sim.step(args.warmup, w.dt)
    sim.kernel_times(reset=True)
    kbuf = torch.zeros(((n + 1023) // 1024) * 1024, dtype=torch.uint8, device="cuda")
    rb = launch.get("react_block", 256)
    ksum = kwave = ksat = 0
    khist = torch.zeros(256, dtype=torch.int64, device="cuda")
    kt_steps = args.steps
    for _ in range(kt_steps):
        sim.step(1, w.dt, flags=mono.STEP_TIMED)
        with torch.cuda.stream(stream):
            sim.get_device_async(mono.FIELD_K, kbuf.data_ptr())
            kk = kbuf.to(torch.int64)
            khist += torch.bincount(kk[:n], minlength=256)[:256]
            ksum += int(kk.sum())
            if launch.get("react_sort", 0):
                # lanes take the nodes of their workgroup in order of k
                kw = kk[:((n + rb - 1) // rb) * rb].view(-1, rb).sort(dim=1).values
            else:
                kw = kk
            kwave += 64 * int(kw.reshape(-1, 64).amax(dim=1).sum())
            ksat += int((kk[:n] == info["k_max"]).sum())
    torch.cuda.synchronize()
    kt = sim.kernel_times()
    # per-launch events cost a few microseconds of their own, which matters for
    # the ~10 us diffusion kernel: its duration is taken from a graph of
    # back-to-back substeps, and the reaction's from the timed window's step
    # time minus the diffusion substeps (the per-launch event figures are
    # reported beside them)
    L = max(sim.info(q)["l"] for q in range(info["n_instances"]))   # substeps per half step
    d_graph_us = 1e3 * sim.time_diffusion(64 * 2 * L)
    sim.close()
    d_event_us = 1e3 * kt["diffusion_ms"] / max(1, kt["diffusion_launches"])
    r_event_us = 1e3 * kt["reaction_ms"] / max(1, kt["reaction_launches"])
    d_us = d_graph_us
    r_us = 1e3 * ms / args.steps - 2 * L * d_us

    # algorithmic work per launch
    P = info["ell_width"]
    by_class = (info["layout"] == mono.LAYOUT_STENCIL and info["row_classes"] > 0
                and launch.get("diff_classes", 1))
    row_bytes = _diff_row_bytes(info, launch, es)
    diff_bytes = n * row_bytes
    # op count of one substep at the library's own initial (resting) state,
    # read from a 4-node simulation
    tiny = mono.Sim.from_workload(W.sheet_tp06(n=2, t_end=0.1), "f64")
    rest = [float(tiny.get(mono.FIELD_STATE0 + j)[0]) for j in range(tiny.info()["n_states"])]
    tiny.close()
    ops = mono.model_flops(W.MODEL_TP06, rest, W.TP06_PARAM_DEFAULT)
    f_model = ops["add"] + ops["mul"] + ops["div"] + ops["exp"] + ops["log"] + ops["sqrt"]
    react_flops = (ksum / kt_steps) * f_model
    diff_total = 2 * L * d_us * 1e-3
    react_total = r_us * 1e-3
    by_rows = by_class and info["grid_rows"] and launch.get("diff_wave_rows", 1)
    tname = "double" if prec == "f64" else "float"
    vpeak = FP64_VECTOR_PEAK_TFLOPS if prec == "f64" else FP32_VECTOR_PEAK_TFLOPS
    # the committed traffic counters were taken in FP32
    tkey = traffic_key if prec == "f32" else None
    launches = info["diff_launches"] or L            # diffusion launches per half step
    fused = launches < L
    if fused:
        # L substeps in `launches` launches of the fused kernel: each reads V,
        # the class ids and writes V once (the substeps in between stay on
        # chip); its per-substep figure is what L unfused launches would move
        per_launch_us = d_us * L / launches
        fused_bytes = n * (2 * es + 2)
        diff_roof = {"kernel": f"k_diff_fused<{tname},{L // launches}>", "bound": "hbm",
                     "achieved": fused_bytes / (per_launch_us * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "bytes_per_row": 2 * es + 2,
                     "substeps_per_launch": L / launches, "launches_per_half_step": launches,
                     "avg_us": per_launch_us, "avg_us_per_substep": d_us,
                     "unfused_equivalent_GBs": diff_bytes / (d_us * 1e-6) / 1e9,
                     "avg_us_per_launch_events": d_event_us,
                     "traffic": _traffic("diffusion", tkey, launch)}
    else:
        diff_roof = {"kernel": ("k_diff_rows" if by_rows else "k_diff_classes" if by_class else
                                "k_diff_stencil" if info["layout"] == mono.LAYOUT_STENCIL
                                else "k_diff_ell") + f"<{tname},{P}>",
                     "bound": "hbm", "achieved": diff_bytes / (d_us * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "bytes_per_row": row_bytes,
                     "avg_us": d_us, "avg_us_per_launch_events": d_event_us,
                     "traffic": _traffic("diffusion", tkey, launch)}
    diff_roof["frac"] = diff_roof["achieved"] / HBM_PEAK_GBS
    react_roof = {"kernel": f"k_ionic<{tname},TP06>", "bound": "alu",
                  "achieved": react_flops / (r_us * 1e-6) / 1e12, "peak": vpeak,
                  "unit": "TFLOP/s", "ops_per_substep": ops, "substeps_per_launch": ksum / kt_steps,
                  "wavefront_efficiency": ksum / kwave if kwave else None, "avg_us": r_us,
                  "avg_us_per_launch_events": r_event_us,
                  "traffic": _traffic("reaction", tkey, launch)}
    react_roof["frac"] = react_roof["achieved"] / vpeak
    # the same launch against the HBM roofline (the bound where k is small)
    rb = n * _react_node_bytes(w, info, es)
    react_roof["hbm"] = {"bytes_per_node": rb / n, "bytes": rb,
                         "achieved": rb / (r_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": rb / (r_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    dominant = react_roof if react_total >= diff_total else diff_roof
    roofline = {k: dominant[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    roofline["kernel"] = dominant["kernel"]
    if dominant is react_roof and prec == "f32":
        roofline["peak_plain_valu"] = FP32_PLAIN_VALU_PEAK_TFLOPS
        roofline["frac_plain_valu"] = react_roof["achieved"] / FP32_PLAIN_VALU_PEAK_TFLOPS

    # accuracy against the FP64 path (itself checked against the FP64 oracle)
    accuracy = None
    if not args.no_accuracy and prec == "f32":
        total = args.warmup + args.steps
        ref = mono.Sim.from_workload(w, "f64", stream=stream.cuda_stream, layout=layout)
        ref.step(total, w.dt)
        v64 = ref.get(mono.FIELD_V)
        l64 = ref.get(mono.FIELD_LAT)
        ref.close()
        both = (l32 > 0) & (l64 > 0)
        accuracy = {"reference": "FP64 path of the same kernels (parity-tested against the "
                                 "FP64 CPU oracle)",
                    "t_ms": total * w.dt,
                    "v_rms_mV": float(np.sqrt(np.mean((v32 - v64) ** 2))),
                    "v_max_mV": float(np.abs(v32 - v64).max()),
                    "lat_max_ms": float(np.abs(l32 - l64)[both].max()) if both.any() else None,
                    "activated_equal": bool(((l32 > 0) == (l64 > 0)).all())}

    # the other legs accompany the default FP32 run
    main_run = args.workload == "slab" and prec == "f32"
    full = None
    if not args.no_full_run and main_run:
        full = full_run(w, stream, launch, layout, not args.no_accuracy)

    adjoint = None
    if not args.no_adjoint and main_run:
        adjoint = adjoint_leg(stream, not args.no_accuracy, not args.no_tune)

    # the same window in FP64, and the batched and tetrahedral workloads
    legs = None
    if not args.no_legs and main_run:
        legs = {}
        legs["fp64"] = other_leg("fp64", w, "f64", stream, args, layout,
                                 wl_name + ", FP64 state and operator")
        wb = W.batched_sheets(precision="f32")
        legs["batched"] = other_leg("batched", wb, "f32", stream, args, mono.LAYOUT_AUTO,
                                    f"batched_tp06_2d: 64 sheets, sides U{{50..400}} seed 4, "
                                    f"{wb.mesh.n_nodes} nodes, log-normal sigma, dt=0.1 ms")
        # the whole 400 ms of all 64 instances as one graph launch
        legs["batched"]["whole_run_one_graph"] = one_graph_run(
            wb, "f32", stream, legs["batched"]["launch"], mono.LAYOUT_AUTO)
        del wb
        wt = W.slab_ischemic_tets(precision="f32", order="rcm")
        legs["tets"] = other_leg("tets", wt, "f32", stream, args, mono.LAYOUT_AUTO,
                                 "slab_tp06_3d_ischemic_tets 201x201x51 (2,060,451 nodes, "
                                 f"{wt.mesh.n_elems:,} linear tetrahedra), RCM node order, "
                                 "dt=0.1 ms, S1+S2")
        del wt

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_steps, args.cpu_steps_1t)

    out = {"metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
           "data": "synthetic",
           "config": {"workload": wl_name, "launch": launch,
                      "nodes": n, "nnz": info["nnz"], "l": info["l"], "dt_ad": info["dt_ad"],
                      "k_max": info["k_max"],
                      "layout": "stencil" if info["layout"] == mono.LAYOUT_STENCIL else "ell",
                      "sim_ms_per_s": w.dt * args.steps / (ms * 1e-3),
                      "row_classes": info["row_classes"],
                      "mean_k": ksum / (n * kt_steps), "k_at_kmax_frac": ksat / (n * kt_steps),
                      "k_histogram": {str(k): int(c) for k, c in enumerate(khist.tolist()) if c},
                      "node_ms_per_s": n * w.dt * args.steps / (ms * 1e-3),
                      "repeats_ms": [t[0] for t in times],
                      "wall_s": wall, "full_run": full},
           "roofline": roofline,
           "kernels": {"diffusion": diff_roof, "reaction": react_roof,
                       "ms_per_step": {"diffusion": diff_total, "reaction": react_total}},
           "accuracy": accuracy, "adjoint": adjoint, "legs": legs, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
