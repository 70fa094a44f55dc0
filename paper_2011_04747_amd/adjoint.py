"""Gradients of a sensor-mismatch loss through the GPU solver, as a
torch.autograd.Function.

The loss is sum_n sum_q (V_q at reaction entry of step n - target[n, q])^2
over a run of `n_steps` outer steps.  Its inputs are the per-node
conductivity scales sigma (which enter the FE stiffness through
(sigma_i + sigma_j)/2 on every edge) and global multipliers of the TP06
conductance rows g_Na, g_CaL, g_Kr, g_Ks, g_K1.  The forward pass runs the
library's taped forward with uniform checkpoints; the backward pass runs the
library's hand-written adjoint.  Everything numerical happens in libmono.
"""
from __future__ import annotations

import numpy as np

from . import mono
from . import workloads as W

# rows of the TP06 parameter block the five multipliers scale
TP06_SCALING_ROWS = (1, 2, 3, 4, 5)      # gNa, gCaL, gKr, gKs, gK1


class AdjointProblem:
    """A workload, a loss target and the run length of the adjoint."""

    def __init__(self, w: W.Workload, target: np.ndarray, n_steps: int, ckpt_every: int = 50,
                 precision: str = "f32", stream=None, replay_k=None):
        if w.model not in (W.MODEL_TP06, W.MODEL_TP06_TYPES):
            raise ValueError("scaling gradients are defined for the TP06 models")
        self.w = w
        self.target = np.ascontiguousarray(target, dtype=np.float64)
        self.n_steps = int(n_steps)
        self.ckpt_every = int(ckpt_every)
        self.precision = precision
        self.stream = stream
        # optional device uint8 tensor (n_steps x n_nodes): hold the reaction
        # substep counts to a given trace (for comparisons at fixed decisions);
        # the library clamps each entry to [1, k_max]
        if replay_k is not None:
            n = w.mesh.n_nodes
            if (getattr(replay_k, "dtype", None) is None or str(replay_k.dtype) != "torch.uint8"
                    or not replay_k.is_cuda or not replay_k.is_contiguous()
                    or replay_k.dim() != 2 or replay_k.shape[0] < self.n_steps
                    or replay_k.shape[1] != n):
                raise ValueError(f"replay_k must be a contiguous uint8 CUDA tensor of shape "
                                 f"(>= {self.n_steps}, {n})")
        self.replay_k = replay_k
        self.sim = None

    def make_sim(self, sigma: np.ndarray, scalings: np.ndarray) -> mono.Sim:
        mesh = self.w.mesh
        m = W.Mesh(mesh.dim, mesh.xyz, mesh.etype, mesh.conn, mesh.D_elem, sigma,
                   mesh.inst_node_off, mesh.inst_elem_off, mesh.grid_shape)
        p = self.w.params.copy()
        for r, c in zip(TP06_SCALING_ROWS, scalings):
            p[r] = p[r] * float(c)
        sim = mono.Sim(m, self.precision, stream=self.stream)
        sim.set_cell_model(self.w.model, p, None, self.w.dt0)
        sim.set_lat_threshold(self.w.lat_threshold)
        for st in self.w.stimuli:
            sim.add_stimulus(st.nodes, st.t_on, st.duration, st.amplitude)
        sim.set_sensors(self.w.sensors, self.target)
        if self.replay_k is not None:
            sim.ktrace(2, None, self.replay_k.data_ptr(), self.replay_k.shape[0], 0)
        return sim


def _autograd():
    import torch

    class MonoAdjointFn(torch.autograd.Function):
        """loss = MonoAdjointFn.apply(sigma, scalings, problem)"""

        @staticmethod
        def forward(ctx, sigma, scalings, problem):
            sg = sigma.detach().to("cpu", torch.float64).numpy()
            sc = scalings.detach().to("cpu", torch.float64).numpy()
            sim = problem.make_sim(sg, sc)
            loss = sim.forward_taped(problem.n_steps, problem.w.dt, problem.ckpt_every)
            ctx.sim = sim
            ctx.sc = sc
            ctx.dev = sigma.device
            return torch.tensor(loss, dtype=torch.float64, device=sigma.device)

        @staticmethod
        def backward(ctx, gout):
            gs, gp = ctx.sim.backward()
            ctx.sim.close()
            ctx.sim = None
            # gp[a] = sum_i p_i[a] dL/dp_i[a]; p_i[a] = c_a base_i[a] gives
            # dL/dc_a = gp[a] / c_a
            gsc = np.array([gp[r] / c for r, c in zip(TP06_SCALING_ROWS, ctx.sc)])
            g = gout.to("cpu", torch.float64)
            return (torch.from_numpy(gs).to(ctx.dev) * g.to(ctx.dev),
                    torch.from_numpy(gsc).to(ctx.dev) * g.to(ctx.dev), None)

    return MonoAdjointFn


_FN = None


def mono_adjoint_fn():
    """The torch.autograd.Function class (created on first use)."""
    global _FN
    if _FN is None:
        _FN = _autograd()
    return _FN
