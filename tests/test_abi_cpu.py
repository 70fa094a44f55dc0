"""Host-side checks of the C interface that need no GPU: the library loads,
exports every entry point its header declares, and rejects bad meshes in
the host assembly before touching the device."""
import os
import re

import numpy as np
import pytest

from paper_2011_04747_amd import mono
from paper_2011_04747_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "mono.h")) as f:
        txt = f.read()
    decl = r"^(?:mono_status|void|const char)\s*\*?\s*(mono_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.M)))


def test_library_exports_every_declared_entry_point():
    L = mono.lib()
    declared = _header_functions()
    assert len(declared) >= 19
    missing = [f for f in declared if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(mono.EXPORTS) == declared


def _desc_create(mesh, **over):
    import ctypes as C
    xyz = np.ascontiguousarray(mesh.xyz, np.float64)
    conn = np.ascontiguousarray(mesh.conn, np.int32)
    D = np.ascontiguousarray(mesh.D_elem, np.float64)
    off = None if mesh.inst_node_off is None else np.ascontiguousarray(mesh.inst_node_off, np.int64)
    f = dict(dim=mesh.dim, n_nodes=mesh.n_nodes, etype=mesh.etype, n_elems=mesh.n_elems,
             n_instances=mesh.n_instances, layout=0, prec=0)
    f.update(over)
    d = mono.MeshDesc(f["dim"], f["n_nodes"], xyz.ctypes.data, f["etype"], f["n_elems"],
                      conn.ctypes.data, D.ctypes.data, None, f["prec"], None, f["n_instances"],
                      None if off is None else off.ctypes.data, f["layout"])
    h = C.c_void_p()
    rc = mono.lib().mono_create_mesh(C.byref(d), C.byref(h))
    return rc, mono.lib().mono_last_error().decode()


def _quad_mesh(nx=4, ny=3):
    xyz, conn, et = W.structured_grid((nx, ny), 0.1)
    D = np.broadcast_to(np.eye(2) * 1e-3, (conn.shape[0], 2, 2)).copy()
    return W.Mesh(2, xyz, et, conn, D)


def test_rejects_bad_descriptions_on_host():
    m = _quad_mesh()
    assert _desc_create(m, dim=4)[0] == -1
    assert _desc_create(m, etype=8)[0] == -1
    assert _desc_create(m, prec=7)[0] == -1
    assert _desc_create(m, layout=9)[0] == -1
    assert _desc_create(m, n_nodes=0)[0] == -1


def test_rejects_out_of_range_index():
    m = _quad_mesh()
    m.conn = m.conn.copy()
    m.conn[2, 1] = m.n_nodes + 5
    rc, msg = _desc_create(m)
    assert rc == -1 and "out of range" in msg


def test_rejects_inverted_element():
    m = _quad_mesh()
    m.conn = m.conn.copy()
    m.conn[0] = m.conn[0][::-1]          # clockwise: negative Jacobian
    rc, msg = _desc_create(m)
    assert rc == -1 and "Jacobian" in msg


def test_rejects_element_joining_instances():
    m = _quad_mesh(4, 4)
    m.inst_node_off = np.array([0, 6, m.n_nodes], np.int64)
    rc, msg = _desc_create(m)
    assert rc == -1 and "instances" in msg


def test_null_handles_are_rejected():
    L = mono.lib()
    assert L.mono_step(None, 1, 0.1, 0) == -1
    assert L.mono_get_info(None, 0, None) == -1
    assert L.mono_sync(None) == -1
    L.mono_destroy(None)


def test_allocator_hook_arguments():
    """mono_set_allocator takes both functions or neither (no simulation exists
    here, so the hook may change)."""
    from paper_2011_04747_amd import mono
    mono.set_allocator(lambda n: 0, lambda p: None)
    mono.set_allocator()
    rc = mono.lib().mono_set_allocator(mono.ALLOC_FN(lambda n, c: None), mono.FREE_FN(), None)
    assert mono.STATUS[rc] == "EINVAL"


def test_nrmse_of_eq4():
    """mono_nrmse (host function of the library): eq. (4) over the entries
    measured in both fields."""
    from paper_2011_04747_amd import mono
    rng = np.random.default_rng(0)
    u = rng.uniform(10.0, 60.0, 1000)
    uh = u + rng.normal(0.0, 0.5, 1000)
    uh[::97] = -1.0                    # unmeasured entries are left out
    keep = uh >= 0
    ref = np.sqrt(np.mean((uh[keep] - u[keep]) ** 2)) / (u[keep].max() - u[keep].min())
    assert mono.nrmse(uh, u) == pytest.approx(ref, rel=1e-12)
    assert mono.nrmse(u, u) == 0.0
    assert np.isnan(mono.nrmse(np.full(3, 5.0), np.full(3, 5.0)))


def test_adjoint_problem_rejects_bad_replay_trace():
    """The autograd problem checks a replayed k-trace before the library sees
    its pointer: dtype, device, contiguity and shape."""
    import torch
    from paper_2011_04747_amd.adjoint import AdjointProblem
    from paper_2011_04747_amd import workloads as W
    w = W.adjoint_slab(shape=(5, 4, 3), t_end=1.0, n_sensors=4)
    tgt = np.zeros((w.n_steps, 4))
    for bad in (torch.zeros((w.n_steps, w.mesh.n_nodes), dtype=torch.uint8),      # host
                torch.zeros((w.n_steps, w.mesh.n_nodes), dtype=torch.int32),
                torch.zeros((w.n_steps, w.mesh.n_nodes + 1), dtype=torch.uint8),
                torch.zeros((w.n_steps - 1, w.mesh.n_nodes), dtype=torch.uint8)):
        with pytest.raises(ValueError):
            AdjointProblem(w, tgt, w.n_steps, replay_k=bad)
