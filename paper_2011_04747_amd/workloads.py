"""Seeded synthetic inputs for the DAETI monodomain solver.

This module only *describes* problems: node coordinates, element
connectivity, per-element diffusion tensors, per-node conductivity and
ionic-parameter fields, stimulus node sets and run lengths.  It contains none
of the solver's arithmetic (no assembly, no time stepping, no cell model), so
that the FP64 CPU oracle and the HIP path can both consume exactly the same
arrays without sharing any numerical code.

Element node ordering (both sides rely on it):
  * line2: x-, x+
  * quad4: (0,0) (1,0) (1,1) (0,1)                        counter-clockwise
  * hex8 : the quad4 face at z-, then the quad4 face at z+
  * tri3 / tet4 (linear simplices): any order with positive orientation

Node numbering of structured grids is lexicographic, x fastest:
  node(ix, iy, iz) = ix + nx*(iy + ny*iz).

The diffusion tensor of every element is D_t*I + (D_l - D_t)*f f^T with f the
unit fibre direction at the element centroid (monodomain eq. 1, tensor D; the
paper's 2D sheets use d0 and the transverse ratio rho the same way, Sec. 3.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# cell-model identifiers (shared vocabulary of both sides' Python wrappers)
MODEL_LINEAR = 0
MODEL_MS = 1
MODEL_TP06 = 2
MODEL_TP06_TYPES = 3    # TP06 with a per-node transmural cell type (7th row)
MODEL_TP06_FIBRO = 4    # TP06 myocytes and passive fibroblasts (class, g_f, E_f rows)

# transmural cell types of MODEL_TP06_TYPES
CELL_EPI = 0
CELL_ENDO = 1
CELL_M = 2
# node classes of MODEL_TP06_FIBRO
NODE_MYOCYTE = 0
NODE_FIBROBLAST = 1
# passive fibroblast membrane (rows 7 and 8 of MODEL_TP06_FIBRO): rate g_f
# [1/ms], a 4 nS membrane conductance over the myocytes' 185 pF (the tissue
# capacitance of the monodomain), and reversal potential E_f [mV]
FIBRO_PARAM_NAMES = ("g_f", "E_f")
FIBRO_PARAM_DEFAULT = (0.0216, -49.6)

ETYPE_LINE2 = 2
ETYPE_TRI3 = 3
ETYPE_QUAD4 = 4
ETYPE_TET4 = 4          # with dim 3
ETYPE_HEX8 = 8

# Per-node TP06 parameter rows (SoA): extracellular K+ and five conductance
# scalings.  Defaults are the published epicardial values (Ko = 5.4 mM,
# scalings 1).
TP06_PARAM_NAMES = ("Ko", "gNa", "gCaL", "gKr", "gKs", "gK1")
TP06_PARAM_DEFAULT = (5.4, 1.0, 1.0, 1.0, 1.0, 1.0)
# Mitchell-Schaeffer parameters (ms), in this row order.
MS_PARAM_NAMES = ("tau_in", "tau_out", "tau_open", "tau_close", "v_gate")
MS_PARAM_DEFAULT = (0.3, 6.0, 120.0, 150.0, 0.13)
LINEAR_PARAM_NAMES = ("g", "E")

# Stimulus amplitudes, dV/dt units (1/ms for Mitchell-Schaeffer, mV/ms for
# TP06): twice the diastolic threshold of each protocol's stimulus region
# (Sec. 3.1: 1 ms pulse at twice diastolic threshold).  The thresholds were
# found by bisection with the FP64 CPU oracle; the script that does so and the
# values it wrote live under tests/golden/ (calibrate_stimulus.py,
# stim_thresholds.json) and a test checks these constants against that file.
STIM_AMP_MS_CABLE = 2.0 * 0.07343750000000002
STIM_AMP_TP06_CORNER = 2.0 * 25.0
STIM_AMP_TP06_PLANAR = 2.0 * 28.28125


@dataclasses.dataclass
class Stimulus:
    nodes: np.ndarray        # int32 node indices
    t_on: float              # ms
    duration: float          # ms
    amplitude: float         # dV/dt units


@dataclasses.dataclass
class Mesh:
    dim: int
    xyz: np.ndarray                  # (n_nodes, dim) float64, cm
    etype: int                       # 2, 4 or 8 nodes per element
    conn: np.ndarray                 # (n_elems, etype) int32
    D_elem: np.ndarray               # (n_elems, dim, dim) float64, cm^2/ms
    sigma: Optional[np.ndarray] = None         # (n_nodes,) conductivity scale
    inst_node_off: Optional[np.ndarray] = None  # (n_inst+1,) int64
    inst_elem_off: Optional[np.ndarray] = None  # (n_inst+1,) int64
    grid_shape: Optional[Tuple[int, ...]] = None

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_instances(self) -> int:
        return 1 if self.inst_node_off is None else len(self.inst_node_off) - 1


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    model: int
    params: Optional[np.ndarray]     # (n_params, n_nodes) float64, SoA
    stimuli: List[Stimulus]
    dt: float                        # ms, outer split step
    t_end: float                     # ms
    dt0: float                       # ms, largest stable cell-model step
    precision: str                   # "f64" or "f32"
    lat_threshold: float
    sensors: Optional[np.ndarray] = None
    extra: dict = dataclasses.field(default_factory=dict)
    init_state: Optional[np.ndarray] = None   # (n_states, n_nodes) SoA, None = published

    @property
    def n_steps(self) -> int:
        return int(round(self.t_end / self.dt))


# ---------------------------------------------------------------------------
# structured grids
# ---------------------------------------------------------------------------
def structured_grid(shape: Tuple[int, ...], h: float | Tuple[float, ...]):
    """Regular grid of Q1 elements: returns (xyz, conn, etype)."""
    dim = len(shape)
    hs = (h,) * dim if np.isscalar(h) else tuple(h)
    axes = [np.arange(n, dtype=np.float64) * hh for n, hh in zip(shape, hs)]
    mg = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # x fastest
    xyz = np.stack([m.reshape(-1) for m in mg], axis=1)
    if dim == 1:
        (nx,) = shape
        i = np.arange(nx - 1)
        conn = np.stack([i, i + 1], axis=1)
        et = ETYPE_LINE2
    elif dim == 2:
        nx, ny = shape
        ix, iy = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
        ix = ix.reshape(-1); iy = iy.reshape(-1)
        n00 = ix + nx * iy
        conn = np.stack([n00, n00 + 1, n00 + 1 + nx, n00 + nx], axis=1)
        et = ETYPE_QUAD4
    elif dim == 3:
        nx, ny, nz = shape
        iz, iy, ix = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1),
                                 np.arange(nx - 1), indexing="ij")
        ix = ix.reshape(-1); iy = iy.reshape(-1); iz = iz.reshape(-1)
        b = ix + nx * (iy + ny * iz)
        pl = nx * ny
        conn = np.stack([b, b + 1, b + 1 + nx, b + nx,
                         b + pl, b + pl + 1, b + pl + 1 + nx, b + pl + nx], axis=1)
        et = ETYPE_HEX8
    else:
        raise ValueError("dim must be 1, 2 or 3")
    return xyz, conn.astype(np.int32), et


def structured_simplices(shape: Tuple[int, ...], h: float):
    """Regular grid split into linear simplices: every square into two
    triangles, every cube into the six tetrahedra around its main diagonal
    (Kuhn / Freudenthal split), all positively oriented.  Returns
    (xyz, conn, etype) with the grid's node numbering."""
    xyz, q1, _ = structured_grid(shape, h)
    if len(shape) == 2:
        n00, n10, n11, n01 = (q1[:, a] for a in range(4))
        conn = np.concatenate([np.stack([n00, n10, n11], 1), np.stack([n00, n11, n01], 1)])
        return xyz, conn.astype(np.int32), ETYPE_TRI3
    if len(shape) != 3:
        raise ValueError("simplices need dim 2 or 3")
    # cube corner with offset bits (bx, by, bz) is hex node
    # 4 bz + [(0,0),(1,0),(1,1),(0,1)].index((bx, by))
    def corner(bx, by, bz):
        return q1[:, 4 * bz + [(0, 0), (1, 0), (1, 1), (0, 1)].index((bx, by))]
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        b = [0, 0, 0]
        path = [corner(*b)]
        for ax in perm:
            b[ax] = 1
            path.append(corner(*b))
        # det [e_p0, e_p0 + e_p1, e_p0 + e_p1 + e_p2] = sign of the permutation
        odd = perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0))
        if odd:
            path[1], path[2] = path[2], path[1]
        tets.append(np.stack(path, 1))
    return xyz, np.concatenate(tets).astype(np.int32), ETYPE_TET4


def _spread_bits(v: np.ndarray, dim: int) -> np.ndarray:
    """Insert dim-1 zero bits after each of the low 63 // dim bits of v."""
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(63 // dim):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(dim * b)
    return out


def morton_codes(xyz: np.ndarray) -> np.ndarray:
    """Z-order (Morton) keys of points: the coordinates scaled by one factor
    (the largest side of the bounding box, so the curve is the same along
    every axis) to the integer range of their share of 63 bits, bits
    interleaved (x lowest)."""
    n, dim = xyz.shape
    bits = 63 // dim
    lo = xyz.min(axis=0)
    span = float((xyz.max(axis=0) - lo).max()) or 1.0
    q = np.floor((xyz - lo) / span * (2.0 ** bits - 1)).astype(np.uint64)
    key = np.zeros(n, np.uint64)
    for d in range(dim):
        key |= _spread_bits(q[:, d], dim) << np.uint64(d)
    return key


def renumber(xyz: np.ndarray, conn: np.ndarray, order: str, seed: int = 0):
    """Node renumbering of a mesh: "grid" keeps it, "random" shuffles it
    (seeded), "rcm" shuffles and then applies reverse Cuthill-McKee on the
    node graph (the bandwidth-reducing order an unstructured mesh would be
    stored in), "morton" shuffles and then sorts the nodes along the Z-order
    curve of their coordinates (a locality order that needs no graph).
    Returns (xyz, conn, new_of_old)."""
    n = xyz.shape[0]
    if order == "grid":
        return xyz, conn, np.arange(n)
    rng = np.random.default_rng(seed)
    new_of_old = rng.permutation(n)
    if order == "rcm":
        import scipy.sparse as sp
        from scipy.sparse.csgraph import reverse_cuthill_mckee
        c = new_of_old[conn].astype(np.int32)
        k = c.shape[1]
        pairs = [(a, b) for a in range(k) for b in range(k) if a != b]
        rows = np.concatenate([c[:, a] for a, _ in pairs])
        cols = np.concatenate([c[:, b] for _, b in pairs])
        g = sp.coo_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(n, n)).tocsr()
        rcm = np.asarray(reverse_cuthill_mckee(g, symmetric_mode=True))   # old(shuffled) at new
        pos = np.empty(n, np.int64)
        pos[rcm] = np.arange(n)
        new_of_old = pos[new_of_old]
    elif order == "morton":
        key = np.empty(n, np.uint64)
        key[new_of_old] = morton_codes(xyz)            # key of each shuffled index
        zs = np.argsort(key, kind="stable")            # shuffled index at new position
        pos = np.empty(n, np.int64)
        pos[zs] = np.arange(n)
        new_of_old = pos[new_of_old]
    elif order != "random":
        raise ValueError("order must be grid, random, rcm or morton")
    xyz2 = np.empty_like(xyz)
    xyz2[new_of_old] = xyz
    return xyz2, new_of_old[conn].astype(np.int32), new_of_old


def centroids(xyz: np.ndarray, conn: np.ndarray) -> np.ndarray:
    return xyz[conn].mean(axis=1)


def fibre_tensor(f: np.ndarray, D_l: float, D_t: float) -> np.ndarray:
    """Per-element tensors D_t I + (D_l - D_t) f f^T for unit fibres f (E, d)."""
    d = f.shape[1]
    return D_t * np.eye(d)[None] + (D_l - D_t) * f[:, :, None] * f[:, None, :]


def angle_fibres(theta: np.ndarray, dim: int) -> np.ndarray:
    f = np.zeros((theta.shape[0], dim))
    f[:, 0] = np.cos(theta)
    if dim > 1:
        f[:, 1] = np.sin(theta)
    return f


def gaussian_random_field(shape: Tuple[int, ...], dx: float, corr_len: float,
                          seed: int) -> np.ndarray:
    """Zero-mean, unit-variance field with covariance exp(-r^2 / (2 l^2)).

    White noise is smoothed by a Gaussian kernel of standard deviation l/sqrt(2)
    (reflecting boundaries) and then standardised.  Returned flat, x fastest.
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape[::-1])                  # index [z][y][x]
    s = corr_len / math.sqrt(2.0) / dx
    g = gaussian_filter(w, sigma=s, mode="reflect")
    g = (g - g.mean()) / g.std()
    return g.reshape(-1)


def lognormal_scale(g: np.ndarray, s: float) -> np.ndarray:
    """exp(s g - s^2/2): unit-mean log-normal scale from a standard field."""
    return np.exp(s * g - 0.5 * s * s)


def _default_params(names_defaults, n_nodes: int) -> np.ndarray:
    return np.tile(np.asarray(names_defaults, dtype=np.float64)[:, None], (1, n_nodes))


def tp06_params(n_nodes: int) -> np.ndarray:
    return _default_params(TP06_PARAM_DEFAULT, n_nodes)


def tp06_types_params(types: np.ndarray) -> np.ndarray:
    """Parameter rows of MODEL_TP06_TYPES: the TP06 defaults plus the cell
    type of each node (CELL_EPI, CELL_ENDO or CELL_M)."""
    types = np.asarray(types)
    return np.vstack([tp06_params(types.size), types.astype(np.float64)[None, :]])


def tp06_fibro_params(classes: np.ndarray) -> np.ndarray:
    """Parameter rows of MODEL_TP06_FIBRO: the TP06 defaults, the node class
    (NODE_MYOCYTE or NODE_FIBROBLAST) and the fibroblast membrane rows."""
    classes = np.asarray(classes)
    n = classes.size
    return np.vstack([tp06_params(n), classes.astype(np.float64)[None, :],
                      _default_params(FIBRO_PARAM_DEFAULT, n)])


def ms_params(n_nodes: int) -> np.ndarray:
    return _default_params(MS_PARAM_DEFAULT, n_nodes)


# ---------------------------------------------------------------------------
# the five workloads (and shrinkable variants with the same structure)
# ---------------------------------------------------------------------------
def cable_ms(n_nodes: int = 101, length: float = 1.0, D: float = 0.001,
             t_end: float = 100.0, dt: float = 0.1, stim_len: float = 0.05,
             amp: Optional[float] = None) -> Workload:
    """1D Mitchell-Schaeffer cable, zero-flux ends, FP64 (the parity case)."""
    h = length / (n_nodes - 1)
    xyz, conn, et = structured_grid((n_nodes,), h)
    De = np.full((conn.shape[0], 1, 1), D)
    mesh = Mesh(1, xyz, et, conn, De, grid_shape=(n_nodes,))
    nodes = np.nonzero(xyz[:, 0] <= stim_len + 1e-12)[0].astype(np.int32)
    a = STIM_AMP_MS_CABLE if amp is None else amp
    return Workload("cable_ms_1d", mesh, MODEL_MS, ms_params(n_nodes),
                    [Stimulus(nodes, 0.0, 2.0, a)], dt, t_end, 0.01, "f64", 0.5)


def _corner_stimulus(xyz: np.ndarray, radius: float, amp: float) -> Stimulus:
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    nodes = np.nonzero(r2 <= radius * radius + 1e-12)[0].astype(np.int32)
    return Stimulus(nodes, 0.0, 1.0, amp)


def sheet_tp06(n: int = 201, dx: float = 0.025, D_l: float = 0.0012,
               D_t: float = 0.0003, theta_max_deg: float = 60.0,
               t_end: float = 500.0, dt: float = 0.1, precision: str = "f64",
               amp: Optional[float] = None) -> Workload:
    """2D TP06 sheet, fibre angle rising linearly 0 -> 60 deg along x."""
    xyz, conn, et = structured_grid((n, n), dx)
    c = centroids(xyz, conn)
    width = (n - 1) * dx
    theta = np.deg2rad(theta_max_deg) * c[:, 0] / width
    De = fibre_tensor(angle_fibres(theta, 2), D_l, D_t)
    mesh = Mesh(2, xyz, et, conn, De, grid_shape=(n, n))
    a = STIM_AMP_TP06_CORNER if amp is None else amp
    return Workload("sheet_tp06_2d", mesh, MODEL_TP06, tp06_params(mesh.n_nodes),
                    [_corner_stimulus(xyz, 0.25, a)], dt, t_end, 0.01,
                    precision, -40.0)


def _slab(shape, dx, D_l, D_t, thickness):
    xyz, conn, et = structured_grid(shape, dx)
    c = centroids(xyz, conn)
    theta = np.deg2rad(-60.0 + 120.0 * c[:, 2] / thickness)
    De = fibre_tensor(angle_fibres(theta, 3), D_l, D_t)
    return Mesh(3, xyz, et, conn, De, grid_shape=tuple(shape))


def _planar_s1(xyz, amp, depth=0.05, t_on=0.0):
    nodes = np.nonzero(xyz[:, 0] <= depth + 1e-12)[0].astype(np.int32)
    return Stimulus(nodes, t_on, 1.0, amp)


def ischemic_zone(xyz: np.ndarray, size_xy: Tuple[float, float], z_mid: float,
                  semi=(0.4, 0.3, 0.25), seed: int = 3) -> np.ndarray:
    """Boolean mask of nodes in a seeded, z-rotated ellipsoid."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.25 * size_xy[0], 0.75 * size_xy[0])
    cy = rng.uniform(0.25 * size_xy[1], 0.75 * size_xy[1])
    ang = rng.uniform(0.0, math.pi)
    dx_ = xyz[:, 0] - cx
    dy_ = xyz[:, 1] - cy
    dz_ = xyz[:, 2] - z_mid
    u = math.cos(ang) * dx_ + math.sin(ang) * dy_
    v = -math.sin(ang) * dx_ + math.cos(ang) * dy_
    return (u / semi[0]) ** 2 + (v / semi[1]) ** 2 + (dz_ / semi[2]) ** 2 <= 1.0


def tp06_paced_state() -> dict:
    """The TP06 states at the end of diastole after 400 beats at a cycle
    length of 1000 ms, for normal tissue and for the ischemic zone's
    parameters ({"normal": (19,), "ischemic": (19,)}), as stored by
    tests/golden/pace_tp06.py (FP64 CPU oracle)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "tests", "golden", "tp06_paced.json")
    with open(path) as f:
        d = json.load(f)
    return {k: np.asarray(d[k]["state"], dtype=np.float64) for k in ("normal", "ischemic")}


def slab_ischemic(shape=(201, 201, 51), dx: float = 0.01, D_l: float = 0.0012,
                  D_t: float = 0.0003, t_end: float = 1000.0, dt: float = 0.1,
                  s2_time: float = 320.0, precision: str = "f32",
                  amp: Optional[float] = None, init: str = "rest") -> Workload:
    """3D TP06 slab with an ischemic ellipsoid, S1 at x=0 and cross-field S2.
    init "rest": the model's published initial state everywhere; "paced":
    the paced steady state of normal and of ischemic tissue
    (tp06_paced_state), the protocol of the paper's tissue runs."""
    thickness = (shape[2] - 1) * dx
    mesh = _slab(shape, dx, D_l, D_t, thickness)
    xyz = mesh.xyz
    p = tp06_params(mesh.n_nodes)
    Lx, Ly = (shape[0] - 1) * dx, (shape[1] - 1) * dx
    isc = ischemic_zone(xyz, (Lx, Ly), 0.5 * thickness,
                        semi=(0.4 * Lx / 2.0, 0.3 * Ly / 2.0, 0.25 * thickness / 0.5))
    p[0, isc] = 8.0           # [K+]o, mM
    p[1, isc] = 0.7           # g_Na scaling
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    s1 = _planar_s1(xyz, a)
    s2n = np.nonzero((xyz[:, 0] <= 0.25 * Lx + 1e-12) &
                     (xyz[:, 1] <= 0.5 * Ly + 1e-12))[0].astype(np.int32)
    s2 = Stimulus(s2n, s2_time, 1.0, a)
    y0 = None
    if init == "paced":
        ps = tp06_paced_state()
        y0 = np.where(isc[None, :], ps["ischemic"][:, None], ps["normal"][:, None])
    elif init != "rest":
        raise ValueError("init must be rest or paced")
    return Workload("slab_tp06_3d_ischemic", mesh, MODEL_TP06, p, [s1, s2], dt,
                    t_end, 0.01, precision, -40.0,
                    extra={"ischemic_nodes": int(isc.sum()), "init": init}, init_state=y0)


def slab_ischemic_tets(shape=(201, 201, 51), dx: float = 0.01, D_l: float = 0.0012,
                       D_t: float = 0.0003, order: str = "rcm", seed: int = 7,
                       t_end: float = 1000.0, dt: float = 0.1, s2_time: float = 320.0,
                       precision: str = "f32", amp: Optional[float] = None) -> Workload:
    """The ischemic TP06 slab on linear tetrahedra (six per grid cube), its
    nodes renumbered as an unstructured mesh would be (`order`, see
    renumber): the 3D workload class of the paper's biventricular runs
    (Sec. 3.3), with the slab's fibres, ischemic zone and stimuli."""
    xyz, conn, et = structured_simplices(shape, dx)
    xyz, conn, _ = renumber(xyz, conn, order, seed)
    thickness = (shape[2] - 1) * dx
    c = centroids(xyz, conn)
    theta = np.deg2rad(-60.0 + 120.0 * c[:, 2] / thickness)
    De = fibre_tensor(angle_fibres(theta, 3), D_l, D_t)
    mesh = Mesh(3, xyz, et, conn, De, grid_shape=None)
    p = tp06_params(mesh.n_nodes)
    Lx, Ly = (shape[0] - 1) * dx, (shape[1] - 1) * dx
    isc = ischemic_zone(xyz, (Lx, Ly), 0.5 * thickness,
                        semi=(0.4 * Lx / 2.0, 0.3 * Ly / 2.0, 0.25 * thickness / 0.5))
    p[0, isc] = 8.0
    p[1, isc] = 0.7
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    s1 = _planar_s1(xyz, a)
    s2n = np.nonzero((xyz[:, 0] <= 0.25 * Lx + 1e-12) &
                     (xyz[:, 1] <= 0.5 * Ly + 1e-12))[0].astype(np.int32)
    s2 = Stimulus(s2n, s2_time, 1.0, a)
    return Workload("slab_tp06_3d_ischemic_tets", mesh, MODEL_TP06, p, [s1, s2], dt,
                    t_end, 0.01, precision, -40.0,
                    extra={"ischemic_nodes": int(isc.sum()), "order": order})


def sheet_planar_tp06(n: int = 501, dx: float = 0.01, D_l: float = 0.0017,
                      ratio: float = 0.25, t_on: float = 50.0, t_end: float = 500.0,
                      dt: float = 0.1, precision: str = "f64",
                      amp: Optional[float] = None) -> Workload:
    """The 2D experiment of Sec. 3.1 on a 5 x 5 cm sheet (n x n nodes at dx):
    fibres along x, d0 = 0.0017 cm^2/ms with transverse ratio 0.25, a 1 ms
    planar stimulus on the left edge at t = 50 ms.  TP06 epicardial cells
    stand in for the O'Hara model."""
    xyz, conn, et = structured_grid((n, n), dx)
    De = fibre_tensor(angle_fibres(np.zeros(conn.shape[0]), 2), D_l, ratio * D_l)
    mesh = Mesh(2, xyz, et, conn, De, grid_shape=(n, n))
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    return Workload("sheet_planar_tp06_2d", mesh, MODEL_TP06, tp06_params(mesh.n_nodes),
                    [_planar_s1(xyz, a, t_on=t_on)], dt, t_end, 0.01, precision, -40.0)


def sheet_transmural_tp06(n_wall: int = 151, n_height: int = 51, dx: float = 0.01,
                          D_l: float = 0.0017, ratio: float = 0.25,
                          layers: Tuple[float, float] = (0.3, 0.6), t_on: float = 0.0,
                          t_end: float = 500.0, dt: float = 0.1, precision: str = "f64",
                          amp: Optional[float] = None) -> Workload:
    """A transmural sheet of ventricular wall: x runs from the endocardium
    (x = 0) to the epicardium, endocardial cells up to layers[0] of the
    thickness, M cells up to layers[1], epicardial cells beyond; fibres
    along y, parallel to the wall surfaces, at the planar sheet's
    conductivities (the wall is crossed transverse to the fibres), and a 1 ms
    planar stimulus on the endocardial edge."""
    xyz, conn, et = structured_grid((n_wall, n_height), dx)
    De = fibre_tensor(angle_fibres(np.full(conn.shape[0], 0.5 * np.pi), 2), D_l, ratio * D_l)
    mesh = Mesh(2, xyz, et, conn, De, grid_shape=(n_wall, n_height))
    depth = xyz[:, 0] / ((n_wall - 1) * dx)
    types = np.where(depth <= layers[0], CELL_ENDO, np.where(depth <= layers[1], CELL_M, CELL_EPI))
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    return Workload("sheet_transmural_tp06_2d", mesh, MODEL_TP06_TYPES, tp06_types_params(types),
                    [_planar_s1(xyz, a, t_on=t_on)], dt, t_end, 0.01, precision, -40.0)


def sheet_fibrotic_tp06(n: int = 251, dx: float = 0.02, d0m: float = 0.002,
                        d0f: float = 0.00066, ratio: float = 0.25, fib_frac: float = 0.10,
                        seed: int = 7, s1_time: float = 50.0, s2_time: float = 200.0,
                        t_end: float = 500.0, dt: float = 0.1, precision: str = "f64",
                        amp: Optional[float] = None) -> Workload:
    """The 2D fibrotic sheet of Sec. 3.2: a square sheet (5 x 5 cm at the
    defaults: 251 x 251 nodes at h = 200 um, the coarsest mesh of Table 1),
    fibres along x, a fraction fib_frac of the nodes drawn uniformly at random
    (seeded) as fibroblasts (passive membrane, MODEL_TP06_FIBRO), the rest
    epicardial TP06 myocytes; conductivity d0m between myocytes and d0f in
    every element that holds a fibroblast node (between fibroblasts and
    between myocytes and fibroblasts), transverse ratio `ratio`; cross-field
    protocol: S1 on the left edge at s1_time, S2 over the lower left quarter
    x <= L/4, y <= L/2 at s2_time, 1 ms each."""
    xyz, conn, et = structured_grid((n, n), dx)
    rng = np.random.default_rng(seed)
    nn = n * n
    fib = np.zeros(nn, bool)
    fib[rng.choice(nn, int(round(fib_frac * nn)), replace=False)] = True
    has_fib = fib[conn].any(axis=1)
    d0 = np.where(has_fib, d0f, d0m)
    f = angle_fibres(np.zeros(conn.shape[0]), 2)
    De = np.einsum("e,eij->eij", d0, fibre_tensor(f, 1.0, ratio))
    mesh = Mesh(2, xyz, et, conn, De, grid_shape=(n, n))
    classes = np.where(fib, NODE_FIBROBLAST, NODE_MYOCYTE)
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    L = (n - 1) * dx
    s1 = _planar_s1(xyz, a, t_on=s1_time)
    s2n = np.nonzero((xyz[:, 0] <= 0.25 * L + 1e-12) & (xyz[:, 1] <= 0.5 * L + 1e-12))[0]
    s2 = Stimulus(s2n.astype(np.int32), s2_time, 1.0, a)
    return Workload("sheet_fibrotic_tp06_2d", mesh, MODEL_TP06_FIBRO, tp06_fibro_params(classes),
                    [s1, s2], dt, t_end, 0.01, precision, -40.0,
                    extra={"fibroblasts": int(fib.sum())})


def batched_sheets(n_inst: int = 64, side_lo: int = 50, side_hi: int = 400,
                   dx: float = 0.025, D_l: float = 0.0012, D_t: float = 0.0003,
                   t_end: float = 400.0, dt: float = 0.1, seed: int = 4,
                   precision: str = "f32", amp: Optional[float] = None) -> Workload:
    """Independent 2D TP06 sheets of seeded uneven sizes, concatenated.

    Instance i has s_x x s_y nodes (each side uniform on side_lo..side_hi), a
    log-normal conductivity field (s = 0.3, correlation length 0.5 cm, seed
    4000+i) and its own g_Na, g_Kr, g_CaL scalings ~ U(0.5, 1.5).
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=(n_inst, 2))
    scal = rng.uniform(0.5, 1.5, size=(n_inst, 3))
    xyzs, conns, Ds, sigmas, params = [], [], [], [], []
    node_off = [0]
    elem_off = [0]
    stim_nodes = []
    a = STIM_AMP_TP06_CORNER if amp is None else amp
    for i in range(n_inst):
        sx, sy = int(sides[i, 0]), int(sides[i, 1])
        xyz, conn, et = structured_grid((sx, sy), dx)
        c = centroids(xyz, conn)
        theta = np.deg2rad(60.0) * c[:, 0] / ((sx - 1) * dx)
        Ds.append(fibre_tensor(angle_fibres(theta, 2), D_l, D_t))
        g = gaussian_random_field((sx, sy), dx, 0.5, 4000 + i)
        sigmas.append(lognormal_scale(g, 0.3))
        p = tp06_params(sx * sy)
        p[1] = scal[i, 0]   # g_Na
        p[3] = scal[i, 1]   # g_Kr
        p[2] = scal[i, 2]   # g_CaL
        params.append(p)
        st = _corner_stimulus(xyz, 0.25, a)
        stim_nodes.append(st.nodes + node_off[-1])
        xyzs.append(xyz)
        conns.append(conn + node_off[-1])
        node_off.append(node_off[-1] + sx * sy)
        elem_off.append(elem_off[-1] + conn.shape[0])
    mesh = Mesh(2, np.concatenate(xyzs), ETYPE_QUAD4, np.concatenate(conns).astype(np.int32),
                np.concatenate(Ds), np.concatenate(sigmas),
                np.asarray(node_off, np.int64), np.asarray(elem_off, np.int64))
    stim = Stimulus(np.concatenate(stim_nodes).astype(np.int32), 0.0, 1.0, a)
    return Workload("batched_tp06_2d", mesh, MODEL_TP06, np.concatenate(params, axis=1),
                    [stim], dt, t_end, 0.01, precision, -40.0,
                    extra={"sides": sides, "scalings": scal})


def adjoint_slab(shape=(101, 101, 26), dx: float = 0.01, D_l: float = 0.0012,
                 D_t: float = 0.0003, t_end: float = 300.0, dt: float = 0.1,
                 n_sensors: int = 512, precision: str = "f32",
                 amp: Optional[float] = None) -> Workload:
    """3D TP06 slab for the adjoint: sensors, perturbed-conductivity target."""
    thickness = (shape[2] - 1) * dx
    mesh = _slab(shape, dx, D_l, D_t, thickness)
    rng = np.random.default_rng(5)
    sensors = np.sort(rng.choice(mesh.n_nodes, size=min(n_sensors, mesh.n_nodes),
                                 replace=False)).astype(np.int32)
    g = gaussian_random_field(tuple(shape), dx, 0.5, 55)
    sigma_target = lognormal_scale(g, 0.1)
    a = STIM_AMP_TP06_PLANAR if amp is None else amp
    return Workload("adjoint_tp06_3d", mesh, MODEL_TP06, tp06_params(mesh.n_nodes),
                    [_planar_s1(mesh.xyz, a)], dt, t_end, 0.01, precision, -40.0,
                    sensors=sensors, extra={"sigma_target": sigma_target,
                                            "ckpt_every": 50})


def random_state(model: int, n_nodes: int, seed: int) -> np.ndarray:
    """Seeded cell states (n_states x n_nodes) spread over each variable's
    physiological range, for single-launch parity checks at full size."""
    rng = np.random.default_rng(seed)
    if model == MODEL_LINEAR:
        return rng.uniform(-90.0, 40.0, (1, n_nodes))
    if model == MODEL_MS:
        return np.vstack([rng.uniform(0.0, 1.0, n_nodes), rng.uniform(0.0, 1.0, n_nodes)])
    y = np.empty((19, n_nodes))
    y[0] = rng.uniform(-90.0, 40.0, n_nodes)            # V, mV
    y[1] = rng.uniform(130.0, 140.0, n_nodes)           # K_i
    y[2] = rng.uniform(6.0, 12.0, n_nodes)              # Na_i
    y[3] = 10 ** rng.uniform(-4.5, -3.0, n_nodes)       # Ca_i
    y[4] = 10 ** rng.uniform(-4.5, -1.0, n_nodes)       # Ca_ss
    y[5] = rng.uniform(0.5, 4.0, n_nodes)               # Ca_SR
    y[6] = rng.uniform(0.5, 1.0, n_nodes)               # Rbar
    y[7:] = rng.uniform(0.0, 1.0, (12, n_nodes))        # gates
    return y
