"""Gauge-misfit calibration through the hand-written adjoint of the step (swe_adjoint).

`Calibration` holds the device arrays of one setup (mesh, replayed dt sequence, gauges,
observations, workspace); `AdjointLoss` exposes its loss to torch.autograd with gradients
with respect to the per-cell Manning n, the bed z and the initial state (h, hu, hv), all in
the mesh's input order.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A
from .solver import Mesh, Solver, _ptr, _stream_handle


class Calibration:
    def __init__(self, mesh: Mesh, dt_seq, gauges, obs, every: int, ckpt_every: int = 50,
                 g=9.81, h_dry=1e-6, inflow_q=None):
        self.mesh = mesh
        dev = mesh.device
        dt_seq = np.asarray(dt_seq, np.float64)
        if dt_seq.ndim != 1 or dt_seq.size < 1:
            raise ValueError("dt_seq must be a non-empty 1-D sequence of time steps")
        self.dt = torch.as_tensor(dt_seq, device=dev)
        self.n_steps = int(self.dt.numel())
        gauges = np.asarray(gauges, np.int64)
        if (gauges.ndim != 1 or gauges.size < 1 or gauges.min() < 0 or
                gauges.max() >= mesh.n_cells or np.unique(gauges).size != gauges.size):
            raise ValueError(f"gauges must be distinct cell ids in [0, {mesh.n_cells})")
        inv = np.empty(mesh.n_cells, np.int64)
        inv[mesh.perm] = np.arange(mesh.n_cells)
        self.gauges = torch.as_tensor(inv[gauges].astype(np.int32), device=dev)
        obs = np.asarray(obs, np.float64).reshape(-1, len(gauges))
        if obs.shape[0] != self.n_steps // every:
            raise ValueError("need one observation row per `every` steps")
        self.obs = torch.as_tensor(obs.ravel(), device=dev)
        self.every, self.ckpt_every = int(every), int(ckpt_every)
        self.g, self.h_dry = g, h_dry
        self.inflow_q = inflow_q
        nbytes = A.swe_adjoint_workspace_bytes(mesh.handle, self.n_steps, self.ckpt_every)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.loss = A.swe_loss(_ptr(self.gauges), len(gauges), self.every, _ptr(self.obs))

    def run(self, n, z, h, hu, hv, stream=None, variant="auto"):
        """J and its gradients (dn, dz, dh, dhu, dhv) as float64 numpy arrays in input order.
        variant: the step kernel of the forward passes ("tiled" also tiles the flux adjoint)."""
        m = self.mesh
        sv = Solver(m, z, n, h, hu, hv, dtype="f64", g=self.g, h_dry=self.h_dry,
                    inflow_q=self.inflow_q, stream=stream, variant=variant)
        t = m.n_cells
        out = [torch.empty(t, dtype=torch.float64, device=m.device) for _ in range(5)]
        grads = A.swe_grads(*[_ptr(o) for o in out])
        j = A.swe_adjoint(m.handle, m.dev, sv.params, sv.state, self.n_steps, _ptr(self.dt),
                          self.loss, self.ckpt_every, grads, _ptr(self.ws), self.ws.numel(),
                          _stream_handle(stream))
        return j, tuple(m.to_input_order(o.cpu().numpy()) for o in out)


class AdjointLoss(torch.autograd.Function):
    """J(n, z, h0, hu0, hv0) of a Calibration; backward returns the adjoint's gradients."""

    @staticmethod
    def forward(ctx, calib: Calibration, n, z, h, hu, hv):
        arr = [t.detach().double().cpu().numpy() for t in (n, z, h, hu, hv)]
        j, grads = calib.run(*arr)
        ctx.grads = [torch.as_tensor(g, dtype=t.dtype, device=t.device)
                     for g, t in zip(grads, (n, z, h, hu, hv))]
        return torch.tensor(j, dtype=torch.float64, device=n.device)

    @staticmethod
    def backward(ctx, grad_out):
        return (None, *[g * grad_out.to(g.dtype) for g in ctx.grads])
