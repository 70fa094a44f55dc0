"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads oracle/liboracle.so (built by oracle/build.py from
oracle/oracle.cpp) and never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same source (the sanitizer build)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

F_V, F_VPREV, F_LAT, F_K, F_STATE0 = 0, 1, 2, 3, 16
DAETI, OSTAR, OST = 0, 1, 2

_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_bp = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def use_library(path):
    """Load another build of the same source (before the first call)."""
    global LIB_PATH
    if _lib is not None and os.path.abspath(path) != os.path.abspath(LIB_PATH):
        raise RuntimeError("the oracle library is already loaded from " + LIB_PATH)
    LIB_PATH = path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("oracle_build", os.path.join(HERE, "build.py"))
            m = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(m)
            m.build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_last_error.restype = C.c_char_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, C.c_int64, _dp, C.c_int, C.c_int64, _ip, _dp, vp,
                                 C.c_int32, vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_nnz.restype = C.c_int64
        L.orc_nnz.argtypes = [vp]
        L.orc_get_matrix.argtypes = [vp, _lp, _ip, _dp, _dp]
        L.orc_set_model.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_double, C.c_double]
        L.orc_add_stimulus.argtypes = [vp, C.c_int64, _ip, C.c_double, C.c_double, C.c_double]
        L.orc_set_method.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.orc_prepare.argtypes = [vp, C.c_double]
        L.orc_info.argtypes = [vp, C.c_int, _dp]
        L.orc_step.argtypes = [vp, C.c_int64, C.c_double]
        L.orc_get_field.argtypes = [vp, C.c_int, _dp]
        L.orc_set_field.argtypes = [vp, C.c_int, _dp]
        L.orc_set_step.argtypes = [vp, C.c_int64]
        L.orc_set_ktrace.argtypes = [vp, C.c_int, vp, vp, C.c_int64]
        L.orc_set_sensors.argtypes = [vp, C.c_int32, _ip, vp, C.c_int64]
        L.orc_set_vclamp.argtypes = [vp, C.c_int]
        L.orc_model_nstates.argtypes = [C.c_int]
        L.orc_model_nparams.argtypes = [C.c_int]
        for f in (L.orc_free_from_total, L.orc_total_from_free):
            f.restype = C.c_double
            f.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_model_init.argtypes = [C.c_int, _dp]
        L.orc_cell_advance.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_double, C.c_int]
        L.orc_cell_rates.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _ip]
        L.orc_tp06_currents.argtypes = [_dp, _dp, _dp]
        L.orc_diffusion_rows.argtypes = [vp, _dp, C.c_double, C.c_int, C.c_int64, _lp, _dp]
        L.orc_reaction_nodes.argtypes = [vp, C.c_int64, C.c_int64, _lp, _dp, _dp, _dp, _ip]
        L.orc_set_target.argtypes = [vp, C.c_int32, _ip, _dp, C.c_int64]
        L.orc_forward_taped.argtypes = [vp, C.c_int64, C.c_double, _dp]
        L.orc_backward.argtypes = [vp, _dp, _dp]
        L.orc_k_rule.argtypes = [C.c_double, C.c_int]
        L.orc_l_rule.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_apd90.argtypes = [C.c_int64, C.c_int64, _dp, C.c_int64, C.c_double, C.c_double,
                                _dp, _dp]
        _lib = L
    return _lib


def set_threads(n):
    """Number of OpenMP threads of the oracle's parallel loops (the OpenMP
    runtime the oracle library is linked against)."""
    import ctypes.util
    lib()
    gomp = C.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    gomp.omp_set_num_threads(int(n))


def get_threads():
    import ctypes.util
    lib()
    gomp = C.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    return int(gomp.omp_get_max_threads())


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """One FP64 CPU simulation of a workload (mesh + cell model + stimuli)."""

    def __init__(self, mesh, model=None, params=None, init_state=None, dt0=0.01,
                 lat_threshold=0.0, stimuli=(), method=DAETI, dvdt_source=0,
                 l_round=0):
        L = lib()
        self.mesh = mesh
        self.n = mesh.n_nodes
        xyz = _f64(mesh.xyz)
        conn = _i32(mesh.conn)
        D = _f64(mesh.D_elem)
        self._keep = [xyz, conn, D]
        sig = None
        if mesh.sigma is not None:
            sig = _f64(mesh.sigma)
            self._keep.append(sig)
        off = None
        ni = 1
        if mesh.inst_node_off is not None:
            off = np.ascontiguousarray(mesh.inst_node_off, dtype=np.int64)
            self._keep.append(off)
            ni = len(off) - 1
        h = L.orc_create(mesh.dim, self.n, xyz, mesh.etype, mesh.n_elems, conn, D,
                         None if sig is None else sig.ctypes.data, ni,
                         None if off is None else off.ctypes.data)
        if not h:
            raise RuntimeError("oracle: " + L.orc_last_error().decode())
        self.h = h
        self.n_inst = ni
        self.model = None
        if model is not None:
            self.set_model(model, params, init_state, dt0, lat_threshold)
        for st in stimuli:
            self.add_stimulus(st.nodes, st.t_on, st.duration, st.amplitude)
        if method != DAETI or dvdt_source or l_round:
            self.set_method(method, dvdt_source, l_round)
        self._ktrace = None

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w.mesh, w.model, w.params, w.init_state, w.dt0, w.lat_threshold, w.stimuli,
                   **kw)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # -- setup ---------------------------------------------------------------
    def set_model(self, model, params=None, init_state=None, dt0=0.01, lat_threshold=0.0):
        L = lib()
        self.model = model
        self.S = L.orc_model_nstates(model)
        self.P = L.orc_model_nparams(model)
        p = None if params is None else _f64(params).reshape(self.P, self.n)
        y0 = None if init_state is None else _f64(init_state).reshape(self.S, self.n)
        self._p, self._y0 = p, y0
        _check(L.orc_set_model(self.h, model, self.P, None if p is None else p.ctypes.data,
                               None if y0 is None else y0.ctypes.data, dt0, lat_threshold))

    def add_stimulus(self, nodes, t_on, duration, amplitude):
        nodes = _i32(nodes)
        _check(lib().orc_add_stimulus(self.h, len(nodes), nodes, t_on, duration, amplitude))

    def set_method(self, method=DAETI, dvdt_source=0, l_round=0):
        _check(lib().orc_set_method(self.h, method, dvdt_source, l_round))

    def prepare(self, dt):
        _check(lib().orc_prepare(self.h, dt))

    def info(self, inst=0):
        out = np.zeros(7)
        _check(lib().orc_info(self.h, inst, out))
        return dict(dt_s=out[0], G_max=out[1], l=int(out[2]), dt_ad=out[3], k_max=int(out[4]),
                    t=out[5], step=int(out[6]))

    def matrix(self):
        """(rowptr, col, val, mass) of the assembled K (with diagonal) and lumped M."""
        nnz = lib().orc_nnz(self.h)
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float64)
        m = np.zeros(self.n, np.float64)
        _check(lib().orc_get_matrix(self.h, rp, col, val, m))
        return rp, col, val, m

    def dense_K(self):
        rp, col, val, m = self.matrix()
        K = np.zeros((self.n, self.n))
        for i in range(self.n):
            K[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
        return K, m

    # -- stepping --------------------------------------------------------------
    def step(self, n_steps, dt):
        _check(lib().orc_step(self.h, int(n_steps), float(dt)))

    def get(self, field):
        out = np.zeros(self.n)
        _check(lib().orc_get_field(self.h, int(field), out))
        return out

    def set(self, field, values):
        _check(lib().orc_set_field(self.h, int(field), _f64(values)))

    def state(self, j):
        return self.get(F_STATE0 + j)

    def set_step(self, step):
        _check(lib().orc_set_step(self.h, int(step)))

    def set_vclamp(self, on):
        _check(lib().orc_set_vclamp(self.h, int(on)))

    def record_k(self, n_steps, with_d=False):
        """Record the k chosen by every node at every step (and dV/dt)."""
        kb = np.zeros((n_steps, self.n), np.uint8)
        db = np.zeros((n_steps, self.n), np.float64) if with_d else None
        self._ktrace = (kb, db)
        _check(lib().orc_set_ktrace(self.h, 1, kb.ctypes.data,
                                    None if db is None else db.ctypes.data, n_steps))
        return kb, db

    def replay_k(self, ktrace):
        kb = np.ascontiguousarray(ktrace, dtype=np.uint8)
        self._ktrace = (kb, None)
        _check(lib().orc_set_ktrace(self.h, 2, kb.ctypes.data, None, kb.shape[0]))

    def ktrace_off(self):
        _check(lib().orc_set_ktrace(self.h, 0, None, None, 0))
        self._ktrace = None

    def diffusion_rows(self, V_in, t0, m, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows))
        _check(lib().orc_diffusion_rows(self.h, _f64(V_in), float(t0), int(m), len(rows), rows, out))
        return out

    def reaction_nodes(self, nstep, rows, y, vprev, lat):
        """Step A on `rows` from states y (S x len(rows)); returns (y, vprev, lat, k)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = _f64(y).copy()
        vp = _f64(vprev).copy()
        la = _f64(lat).copy()
        k = np.zeros(len(rows), np.int32)
        _check(lib().orc_reaction_nodes(self.h, int(nstep), len(rows), rows, y, vp, la, k))
        return y, vp, la, k

    # -- adjoint ----------------------------------------------------------------
    def set_target(self, nodes, target):
        """Loss sensors and targets (n_steps x len(nodes)), sampled at reaction entry."""
        nodes = _i32(nodes)
        t = _f64(target)
        self._target = (nodes, t)
        _check(lib().orc_set_target(self.h, len(nodes), nodes, t.reshape(-1), t.shape[0]))

    def forward_taped(self, n_steps, dt):
        out = np.zeros(1)
        _check(lib().orc_forward_taped(self.h, int(n_steps), float(dt), out))
        return float(out[0])

    def backward(self):
        """(dL/dsigma per node, dL/d(common multiplier of each parameter row))."""
        gs = np.zeros(self.n)
        gp = np.zeros(self.P)
        _check(lib().orc_backward(self.h, gs, gp))
        return gs, gp

    def record_sensors(self, nodes, n_steps):
        nodes = _i32(nodes)
        buf = np.zeros((n_steps, len(nodes)), np.float64)
        self._sens = (nodes, buf)
        _check(lib().orc_set_sensors(self.h, len(nodes), nodes, buf.ctypes.data, n_steps))
        return buf


# -- cell-level helpers ----------------------------------------------------------
def model_nstates(model):
    return lib().orc_model_nstates(model)


def model_init(model):
    y = np.zeros(model_nstates(model))
    lib().orc_model_init(model, y)
    return y


def cell_advance(model, params, y, k, dt, vclamp=False):
    y = _f64(y).copy()
    _check(lib().orc_cell_advance(model, _f64(params), y, int(k), float(dt), int(vclamp)))
    return y


def cell_rates(model, params, y):
    S = model_nstates(model)
    rate, inf, tau = np.zeros(S), np.zeros(S), np.zeros(S)
    gate = np.zeros(S, np.int32)
    _check(lib().orc_cell_rates(model, _f64(params), _f64(y), rate, inf, tau, gate))
    return rate, inf, tau, gate.astype(bool)


TP06_CURRENTS = ("INa", "IK1", "Ito", "IKr", "IKs", "ICaL", "INaCa", "INaK", "IpCa", "IpK",
                 "IbNa", "IbCa", "Irel", "Iup", "Ileak", "Ixfer", "Iion")


def tp06_currents(params, y):
    out = np.zeros(17)
    _check(lib().orc_tp06_currents(_f64(params), _f64(y), out))
    return dict(zip(TP06_CURRENTS, out))


def buffer_free_from_total(total, B, K):
    """Free concentration of an instantaneously buffered pool (TP06 calcium)."""
    return lib().orc_free_from_total(float(total), float(B), float(K))


def buffer_total_from_free(c, B, K):
    return lib().orc_total_from_free(float(c), float(B), float(K))


def k_rule(dvdt, k_max):
    return lib().orc_k_rule(float(dvdt), int(k_max))


def l_rule(dt, dt_s, l_round=0):
    return lib().orc_l_rule(float(dt), float(dt_s), int(l_round))


def apd90(samples, dt, thr, step0=0):
    """APD90 and upstroke time per node from reaction-entry samples
    (steps x nodes, sample n taken at (step0 + n) dt + dt/2); see orc_apd90
    in oracle.cpp for the definition.  Returns (apd, tup), -1 where not
    measured."""
    V = np.ascontiguousarray(samples, np.float64)
    steps, ns = V.shape
    apd = np.zeros(ns, np.float64)
    tup = np.zeros(ns, np.float64)
    _check(lib().orc_apd90(steps, ns, V, int(step0), float(dt), float(thr), apd, tup))
    return apd, tup
