"""Gradients of a sensor-mismatch loss through the GPU solver, as a
torch.autograd.Function.

The loss is sum_n sum_q (V_q at reaction entry of step n - target[n, q])^2
over a run of `n_steps` outer steps.  Its inputs are the per-node
conductivity scales sigma (which enter the FE stiffness through
(sigma_i + sigma_j)/2 on every edge) and global multipliers of the TP06
conductance rows g_Na, g_CaL, g_Kr, g_Ks, g_K1.  The forward pass runs the
library's taped forward with uniform checkpoints; the backward pass runs the
library's hand-written adjoint.  Everything numerical happens in libmono,
including the chain rule through the multipliers: torch supplies device
memory (sigma, the multipliers, the loss and gradient outputs) and streams.
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

    def make_sim(self, sigma_device: int, scalings_device: int) -> mono.Sim:
        """A simulation of the problem with the conductivity scales and the
        row multipliers read from device addresses (n_nodes and 5 FP64
        values, ready when called)."""
        sim = mono.Sim(self.w.mesh, self.precision, stream=self.stream,
                       sigma_device=sigma_device)
        sim.set_cell_model(self.w.model, self.w.params, None, self.w.dt0)
        sim.set_param_scalings(TP06_SCALING_ROWS, scalings_device)
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
            n = problem.w.mesh.n_nodes
            if (not sigma.is_cuda or not scalings.is_cuda or sigma.shape != (n,)
                    or scalings.shape != (len(TP06_SCALING_ROWS),)):
                raise ValueError(f"sigma ({n},) and scalings ({len(TP06_SCALING_ROWS)},) "
                                 f"must be CUDA tensors")
            sg = sigma.detach().to(torch.float64).contiguous()
            sc = scalings.detach().to(torch.float64).contiguous()
            # the library reads both on its own stream
            torch.cuda.current_stream(sigma.device).synchronize()
            sim = problem.make_sim(sg.data_ptr(), sc.data_ptr())
            loss = torch.empty((), dtype=torch.float64, device=sigma.device)
            sim.forward_taped_device(problem.n_steps, problem.w.dt, problem.ckpt_every,
                                     loss.data_ptr())
            ctx.sim = sim
            ctx.dev = sigma.device
            return loss

        @staticmethod
        def backward(ctx, gout):
            n = ctx.sim.n
            gs = torch.empty(n, dtype=torch.float64, device=ctx.dev)
            gsc = torch.empty(len(TP06_SCALING_ROWS), dtype=torch.float64, device=ctx.dev)
            ctx.sim.backward_device(gs.data_ptr(), gsc.data_ptr())
            ctx.sim.close()
            ctx.sim = None
            g = gout.to(device=ctx.dev, dtype=torch.float64)
            return gs * g, gsc * g, None

    return MonoAdjointFn


_FN = None


def mono_adjoint_fn():
    """The torch.autograd.Function class (created on first use)."""
    global _FN
    if _FN is None:
        _FN = _autograd()
    return _FN
