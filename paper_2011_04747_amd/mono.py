"""Thin ctypes binding of libmono (include/mono.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies streams and device buffers where a device pointer is asked
for.  Importing this module does not load the library; the first use does,
and raises if libmono.so has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmono.so")

F64, F32 = 0, 1
LAYOUT_AUTO, LAYOUT_ELL, LAYOUT_STENCIL = 0, 1, 2
FIELD_V, FIELD_VPREV, FIELD_LAT, FIELD_K, FIELD_APD, FIELD_TUP, FIELD_STATE0 = 0, 1, 2, 3, 4, 5, 16
DAETI, OSTAR, OST = 0, 1, 2
DEBUG_KTRACE, DEBUG_VCLAMP, DEBUG_FORCE_L, DEBUG_STATS, DEBUG_STATS_ENABLE = 1, 2, 3, 4, 5
DEBUG_KTIMES = 6
DEBUG_TIME_DIFFUSION = 7
STEP_EAGER, STEP_TIMED, STEP_CAPTURE = 1, 2, 4
CKPT_UNIFORM, CKPT_BINOMIAL = 0, 1

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSUPPORTED",
          -6: "ENONFINITE"}

# exported entry points (include/mono.h); tests check every one is present
EXPORTS = ("mono_create_mesh", "mono_set_cell_model", "mono_set_lat_threshold",
           "mono_add_stimulus", "mono_set_method", "mono_step", "mono_get_state",
           "mono_get_state_device_async", "mono_set_state", "mono_set_time_level",
           "mono_prepare", "mono_get_info", "mono_estimate_lambda", "mono_set_stream",
           "mono_sync", "mono_destroy", "mono_last_error", "mono_apply_phase", "mono_debug",
           "mono_model_flops", "mono_set_launch", "mono_get_launch",
           "mono_model_substep_host", "mono_model_vjp_host", "mono_set_sensors",
           "mono_forward_taped", "mono_backward", "mono_sample_sensors", "mono_set_allocator",
           "mono_track_apd", "mono_nrmse", "mono_set_checkpointing", "mono_checkpoint_info",
           "mono_checkpoint_plan", "mono_sample_sensors_noalloc", "mono_set_param_scalings",
           "mono_forward_taped_device", "mono_backward_device")


class MonoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("xyz", C.c_void_p),
                ("etype", C.c_int32), ("n_elems", C.c_int64), ("conn", C.c_void_p),
                ("D_elem", C.c_void_p), ("sigma_node", C.c_void_p), ("prec", C.c_int32),
                ("stream", C.c_void_p), ("n_instances", C.c_int32),
                ("inst_node_off", C.c_void_p), ("layout", C.c_int32),
                ("sigma_device", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("dt_s", C.c_double), ("G_max", C.c_double), ("lambda_est", C.c_double),
                ("dt_ad", C.c_double), ("dt", C.c_double), ("t", C.c_double),
                ("step", C.c_int64), ("nnz", C.c_int64), ("l", C.c_int32), ("k_max", C.c_int32),
                ("layout", C.c_int32), ("n_instances", C.c_int32), ("n_states", C.c_int32),
                ("ell_width", C.c_int32), ("row_classes", C.c_int32),
                ("grid_rows", C.c_int32), ("diff_fused", C.c_int32),
                ("diff_launches", C.c_int32)]


class Launch(C.Structure):
    _fields_ = [("diff_block", C.c_int32), ("diff_rows_per_lane", C.c_int32),
                ("diff_xcd_remap", C.c_int32), ("react_block", C.c_int32),
                ("graph_steps", C.c_int32), ("react_sort", C.c_int32),
                ("diff_classes", C.c_int32), ("diff_wave_rows", C.c_int32),
                ("diff_fuse", C.c_int32), ("diff_fuse_planes", C.c_int32)]


class KTrace(C.Structure):
    _fields_ = [("mode", C.c_int32), ("record", C.c_void_p), ("replay", C.c_void_p),
                ("n_steps", C.c_int64), ("base_step", C.c_int64)]


_lib = None


# device-memory hook of mono_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator_refs = None   # keeps the installed callbacks alive


def set_allocator(alloc=None, free=None):
    """Route the library's device allocations through alloc(nbytes) -> int
    pointer and free(ptr) (both Python callables), or back to hipMalloc /
    hipFree with no arguments.  Only while no simulation exists."""
    global _allocator_refs
    if alloc is None and free is None:
        _check(lib().mono_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator_refs = None
        return
    fa = ALLOC_FN(lambda nbytes, ctx: int(alloc(int(nbytes))) or None)
    ff = FREE_FN(lambda ptr, ctx: free(int(ptr)))
    _check(lib().mono_set_allocator(fa, ff, None))
    _allocator_refs = (fa, ff)


def use_torch_allocator():
    """Let torch's caching allocator own the library's device memory."""
    import torch
    dev = torch.cuda.current_device()
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev),
                  torch.cuda.caching_allocator_delete)


def lib():
    """Load libmono.so (raises if it is missing: the HIP path is the only path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run "
                              "python paper_2011_04747_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "mono_create_mesh": [C.POINTER(MeshDesc), C.POINTER(vp)],
            "mono_set_cell_model": [vp, i32, i32, vp, vp, dbl],
            "mono_set_lat_threshold": [vp, dbl],
            "mono_add_stimulus": [vp, i64, vp, dbl, dbl, dbl],
            "mono_set_method": [vp, i32, i32, i32],
            "mono_step": [vp, i64, dbl, C.c_uint32],
            "mono_get_state": [vp, i32, vp, i64],
            "mono_get_state_device_async": [vp, i32, vp],
            "mono_set_state": [vp, i32, vp, i64],
            "mono_set_time_level": [vp, i64],
            "mono_prepare": [vp, dbl],
            "mono_get_info": [vp, i32, C.POINTER(Info)],
            "mono_estimate_lambda": [vp, i32],
            "mono_set_stream": [vp, vp],
            "mono_sync": [vp],
            "mono_apply_phase": [vp, i32, i64, i32],
            "mono_debug": [vp, i32, vp],
            "mono_model_flops": [i32, vp, vp, vp],
            "mono_model_substep_host": [i32, vp, vp, dbl, i32],
            "mono_model_vjp_host": [i32, vp, vp, dbl, i32, vp, vp],
            "mono_set_sensors": [vp, i32, vp, vp, i64],
            "mono_forward_taped": [vp, i64, dbl, i32, vp],
            "mono_backward": [vp, vp, vp],
            "mono_sample_sensors": [vp, i64, dbl, vp],
            "mono_set_launch": [vp, C.POINTER(Launch)],
            "mono_get_launch": [vp, C.POINTER(Launch)],
            "mono_set_allocator": [ALLOC_FN, FREE_FN, vp],
            "mono_track_apd": [vp, i32],
            "mono_nrmse": [vp, vp, i64, vp],
            "mono_set_checkpointing": [vp, i32, i32],
            "mono_checkpoint_info": [vp, vp],
            "mono_checkpoint_plan": [i64, i32, vp],
            "mono_sample_sensors_noalloc": [vp, i64, dbl, vp],
            "mono_set_param_scalings": [vp, i32, vp, vp],
            "mono_forward_taped_device": [vp, i64, dbl, i32, vp],
            "mono_backward_device": [vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.mono_destroy.argtypes = [vp]
        L.mono_destroy.restype = None
        L.mono_last_error.argtypes = []
        L.mono_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MonoError(rc, lib().mono_last_error().decode())


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def nrmse(u_hat, u):
    """Eq. (4): sqrt(mean (u_hat - u)^2) / (max u - min u) over the entries
    where both values are measured (non-negative); NaN if none or no range."""
    a = _c(u_hat, np.float64)
    b = _c(u, np.float64)
    assert a.shape == b.shape and a.ndim == 1
    out = np.zeros(1, np.float64)
    _check(lib().mono_nrmse(a.ctypes.data, b.ctypes.data, a.size, out.ctypes.data))
    return float(out[0])


def model_flops(model, state, params):
    """Operation counts of one cell-model substep at `state` (host-side count
    on the kernel's own model code): dict add, mul, div, exp, log, sqrt, cmp."""
    y = _c(state, np.float64)
    p = _c(params, np.float64)
    out = np.zeros(7, np.int64)
    _check(lib().mono_model_flops(int(model), y.ctypes.data, p.ctypes.data, out.ctypes.data))
    return dict(zip(("add", "mul", "div", "exp", "log", "sqrt", "cmp"), (int(v) for v in out)))


def model_substep_host(model, state, params, h, clamp=False):
    """One substep of the kernel's model code, evaluated on the host in FP64."""
    y = np.array(state, dtype=np.float64)
    p = _c(params, np.float64)
    _check(lib().mono_model_substep_host(int(model), y.ctypes.data, p.ctypes.data, float(h),
                                         int(clamp)))
    return y


def model_vjp_host(model, state, params, h, lam, clamp=False):
    """(dF/dy)^T lam and (dF/dp)^T lam of one substep, host FP64."""
    y = _c(state, np.float64)
    p = _c(params, np.float64)
    l = np.array(lam, dtype=np.float64)
    gp = np.zeros(len(p), np.float64)
    _check(lib().mono_model_vjp_host(int(model), y.ctypes.data, p.ctypes.data, float(h),
                                     int(clamp), l.ctypes.data, gp.ctypes.data))
    return l, gp


class Sim:
    """One monodomain simulation on the GPU (a handle of libmono)."""

    def __init__(self, mesh, precision: str = "f64", stream=None, layout: int = LAYOUT_AUTO,
                 sigma_device=None):
        """sigma_device: address of n_nodes FP64 conductivity scales in device
        memory, used instead of mesh.sigma (the library copies them for its
        host-side assembly)."""
        L = lib()
        self.n = mesh.n_nodes
        self.precision = precision
        xyz = _c(mesh.xyz, np.float64)
        conn = _c(mesh.conn, np.int32)
        D = _c(mesh.D_elem, np.float64)
        sig = None if mesh.sigma is None else _c(mesh.sigma, np.float64)
        off = None if mesh.inst_node_off is None else _c(mesh.inst_node_off, np.int64)
        self.stream = stream
        if sigma_device is not None:
            sig_ptr, on_dev = int(sigma_device), 1
        else:
            sig_ptr, on_dev = (None if sig is None else sig.ctypes.data), 0
        d = MeshDesc(mesh.dim, self.n, xyz.ctypes.data, mesh.etype, mesh.n_elems,
                     conn.ctypes.data, D.ctypes.data, sig_ptr,
                     F64 if precision == "f64" else F32,
                     None if stream is None else int(stream), mesh.n_instances,
                     None if off is None else off.ctypes.data, layout, on_dev)
        h = C.c_void_p()
        _check(L.mono_create_mesh(C.byref(d), C.byref(h)))
        self.h = h
        self.n_instances = mesh.n_instances
        self.model = None

    @classmethod
    def from_workload(cls, w, precision: Optional[str] = None, stream=None,
                      layout: int = LAYOUT_AUTO, with_stimuli: bool = True):
        s = cls(w.mesh, precision or w.precision, stream, layout)
        s.set_cell_model(w.model, w.params, w.init_state, w.dt0)
        s.set_lat_threshold(w.lat_threshold)
        if with_stimuli:
            for st in w.stimuli:
                s.add_stimulus(st.nodes, st.t_on, st.duration, st.amplitude)
        return s

    def close(self):
        if getattr(self, "h", None):
            lib().mono_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup -------------------------------------------------------------------
    def set_cell_model(self, model, params=None, init_state=None, dt0=0.01):
        p = None if params is None else _c(params, np.float64)
        y = None if init_state is None else _c(init_state, np.float64)
        npar = 0 if p is None else p.shape[0]
        _check(lib().mono_set_cell_model(self.h, model, npar, None if p is None else p.ctypes.data,
                                         None if y is None else y.ctypes.data, dt0))
        self.model = model

    def set_lat_threshold(self, v):
        _check(lib().mono_set_lat_threshold(self.h, float(v)))

    def add_stimulus(self, nodes, t_on, duration, amplitude):
        nodes = _c(nodes, np.int32)
        _check(lib().mono_add_stimulus(self.h, len(nodes), nodes.ctypes.data, float(t_on),
                                       float(duration), float(amplitude)))

    def set_method(self, method=DAETI, dvdt_source=0, l_round=0):
        _check(lib().mono_set_method(self.h, method, dvdt_source, l_round))

    def prepare(self, dt):
        _check(lib().mono_prepare(self.h, float(dt)))

    # -- stepping ----------------------------------------------------------------
    def step(self, n_steps, dt, flags=0):
        _check(lib().mono_step(self.h, int(n_steps), float(dt), int(flags)))

    def sync(self):
        _check(lib().mono_sync(self.h))

    def apply_phase(self, phase, step, m=0):
        _check(lib().mono_apply_phase(self.h, int(phase), int(step), int(m)))

    def get(self, field):
        out = np.zeros(self.n, np.float64)
        _check(lib().mono_get_state(self.h, int(field), out.ctypes.data, self.n))
        return out

    def state(self, j):
        return self.get(FIELD_STATE0 + j)

    def get_device_async(self, field, dst_ptr):
        _check(lib().mono_get_state_device_async(self.h, int(field), C.c_void_p(int(dst_ptr))))

    def set(self, field, values):
        v = _c(values, np.float64)
        assert v.shape == (self.n,)
        _check(lib().mono_set_state(self.h, int(field), v.ctypes.data, self.n))

    def set_time_level(self, step):
        _check(lib().mono_set_time_level(self.h, int(step)))

    def track_apd(self, on=True):
        """Start (and reset) or stop APD90 tracking (FIELD_APD, FIELD_TUP)."""
        _check(lib().mono_track_apd(self.h, 1 if on else 0))

    def info(self, inst=0):
        i = Info()
        _check(lib().mono_get_info(self.h, int(inst), C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def estimate_lambda(self, iters=100):
        _check(lib().mono_estimate_lambda(self.h, int(iters)))

    def launch(self):
        c = Launch()
        _check(lib().mono_get_launch(self.h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in Launch._fields_}

    def set_launch(self, **kw):
        cur = self.launch()
        cur.update(kw)
        c = Launch(*(int(cur[k]) for k, _ in Launch._fields_))
        _check(lib().mono_set_launch(self.h, C.byref(c)))

    def set_stream(self, stream):
        _check(lib().mono_set_stream(self.h, C.c_void_p(int(stream))))

    # -- adjoint -----------------------------------------------------------------
    def set_sensors(self, nodes, target):
        """Loss sensors and targets (n_steps x len(nodes)) sampled at reaction entry."""
        nodes = _c(nodes, np.int32)
        t = _c(target, np.float64)
        _check(lib().mono_set_sensors(self.h, len(nodes), nodes.ctypes.data, t.ctypes.data,
                                      t.shape[0]))

    def sample_sensors(self, n_steps, dt, n_sensors):
        """Step and return V at the sensors at reaction entry (n_steps x n_sensors)."""
        out = np.zeros((int(n_steps), int(n_sensors)))
        _check(lib().mono_sample_sensors(self.h, int(n_steps), float(dt), out.ctypes.data))
        return out

    def sample_sensors_noalloc(self, n_steps, dt, n_sensors):
        """sample_sensors staged in the library's static device buffer (no
        device allocation; n_steps x n_sensors <= 524288)."""
        out = np.zeros((int(n_steps), int(n_sensors)))
        _check(lib().mono_sample_sensors_noalloc(self.h, int(n_steps), float(dt),
                                                 out.ctypes.data))
        return out

    def forward_taped(self, n_steps, dt, ckpt_every=50):
        out = np.zeros(1)
        _check(lib().mono_forward_taped(self.h, int(n_steps), float(dt), int(ckpt_every),
                                        out.ctypes.data))
        return float(out[0])

    def set_checkpointing(self, schedule="uniform", max_snapshots=0):
        """Checkpoint schedule of the next forward_taped: "uniform" or
        "binomial" within max_snapshots snapshot buffers."""
        code = {"uniform": CKPT_UNIFORM, "binomial": CKPT_BINOMIAL}[schedule]
        _check(lib().mono_set_checkpointing(self.h, code, int(max_snapshots)))

    def checkpoint_info(self):
        out = np.zeros(6, np.int64)
        _check(lib().mono_checkpoint_info(self.h, out.ctypes.data))
        return {"schedule": ("uniform", "binomial")[int(out[0])], "snapshots": int(out[1]),
                "segments": int(out[2]), "advances": int(out[3]),
                "snapshot_bytes": int(out[4]), "tape_bytes": int(out[5])}

    def set_param_scalings(self, rows, scalings_device):
        """Scale parameter rows `rows` by n FP64 values at a device address."""
        r = _c(rows, np.int32)
        _check(lib().mono_set_param_scalings(self.h, len(r), r.ctypes.data,
                                             C.c_void_p(int(scalings_device))))

    def forward_taped_device(self, n_steps, dt, ckpt_every, loss_device):
        """forward_taped with the loss written to a device address (FP64)."""
        _check(lib().mono_forward_taped_device(self.h, int(n_steps), float(dt), int(ckpt_every),
                                               C.c_void_p(int(loss_device))))

    def backward_device(self, grad_sigma_device=None, grad_scalings_device=None):
        """backward with dL/dsigma and dL/d(scalings) written to device addresses."""
        _check(lib().mono_backward_device(
            self.h, None if grad_sigma_device is None else C.c_void_p(int(grad_sigma_device)),
            None if grad_scalings_device is None else C.c_void_p(int(grad_scalings_device))))

    def backward(self, n_params=None):
        """(dL/dsigma per node, derivative for a common multiplier of each parameter row)."""
        gs = np.zeros(self.n)
        gp = np.zeros(16)
        _check(lib().mono_backward(self.h, gs.ctypes.data, gp.ctypes.data))
        P = n_params if n_params is not None else {0: 2, 1: 5, 2: 6, 3: 7, 4: 9}[self.model]
        return gs, gp[:P]

    # -- test hooks --------------------------------------------------------------
    def ktrace(self, mode, record_ptr=None, replay_ptr=None, n_steps=0, base_step=0):
        kt = KTrace(int(mode), None if record_ptr is None else int(record_ptr),
                    None if replay_ptr is None else int(replay_ptr), int(n_steps), int(base_step))
        _check(lib().mono_debug(self.h, DEBUG_KTRACE, C.byref(kt)))
        self._kt = kt

    def vclamp(self, on):
        v = C.c_int32(int(on))
        _check(lib().mono_debug(self.h, DEBUG_VCLAMP, C.byref(v)))

    def force_l(self, l):
        v = C.c_int32(int(l))
        _check(lib().mono_debug(self.h, DEBUG_FORCE_L, C.byref(v)))

    def stats_enable(self, on=True):
        v = C.c_int32(int(on))
        _check(lib().mono_debug(self.h, DEBUG_STATS_ENABLE, C.byref(v)))

    def stats(self):
        """(sum k, sum over wavefronts of 64*max k, node-steps, node-steps at k_max)."""
        out = (C.c_int64 * 4)()
        _check(lib().mono_debug(self.h, DEBUG_STATS, out))
        return tuple(out)

    def kernel_times(self, reset=False):
        """Per-class kernel time of STEP_TIMED steps:
        {diffusion_ms, diffusion_launches, reaction_ms, reaction_launches}."""
        out = (C.c_double * 5)()
        out[4] = 1.0 if reset else 0.0
        _check(lib().mono_debug(self.h, DEBUG_KTIMES, out))
        return dict(diffusion_ms=out[0], diffusion_launches=int(out[1]),
                    reaction_ms=out[2], reaction_launches=int(out[3]))

    def time_diffusion(self, repetitions=384):
        """Mean ms of one diffusion substep over `repetitions` (even) substeps
        replayed as one HIP graph; advances the potential by them."""
        out = (C.c_double * 2)()
        out[0] = float(repetitions)
        _check(lib().mono_debug(self.h, DEBUG_TIME_DIFFUSION, out))
        return out[1]


def checkpoint_plan_advances(n_segments, max_snapshots):
    """Whole-segment forward advances of the binomial checkpoint plan (host)."""
    out = np.zeros(1, np.int64)
    _check(lib().mono_checkpoint_plan(int(n_segments), int(max_snapshots), out.ctypes.data))
    return int(out[0])
