"""Gauge-misfit calibration through the hand-written adjoint of the step (swe_adjoint).

`Calibration` holds the device arrays of one setup (mesh, replayed dt sequence, gauges,
observations, workspace, and the state, bed and roughness buffers the adjoint reads), all
allocated once; `AdjointLoss` exposes its loss to torch.autograd with gradients with respect to
the per-cell Manning n, the bed z and the initial state (h, hu, hv), in the mesh's input order.
Device tensors stay on the device: they are permuted into mesh order and the gradients back
into input order by gathers on the GPU, so a call moves nothing through the host but the loss.
"""
from __future__ import annotations

import contextlib
import ctypes as C

import numpy as np
import torch

from . import _abi as A
from .solver import Mesh, _ptr, _stream_handle


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
        self._q = np.ascontiguousarray(inflow_q if inflow_q is not None else [], np.float64)
        nbytes = A.swe_adjoint_workspace_bytes(mesh.handle, self.n_steps, self.ckpt_every)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.loss = A.swe_loss(_ptr(self.gauges), len(gauges), self.every, _ptr(self.obs))
        # mesh cell i is input cell perm[i]: gathers by perm go to mesh order, scatters back
        self.perm = torch.as_tensor(mesh.perm.astype(np.int64), device=dev)
        t = mesh.n_cells
        # z, n, h, hu, hv in mesh order, and the five gradients (mesh order, then input order)
        self.fields = torch.empty((5, t), dtype=torch.float64, device=dev)
        self.grad_mesh = torch.empty((5, t), dtype=torch.float64, device=dev)
        self.grads = A.swe_grads(*[_ptr(self.grad_mesh[k]) for k in range(5)])
        f = self.fields
        self.state = A.swe_state((C.c_void_p * 2)(f[2].data_ptr(), 0),
                                 (C.c_void_p * 2)(f[3].data_ptr(), 0),
                                 (C.c_void_p * 2)(f[4].data_ptr(), 0),
                                 _ptr(f[0]), _ptr(f[1]), None, None, 0, 0)
        self._variant = None
        self.params = None

    def _params(self, variant: str):
        if self._variant != variant:
            self.params = A.swe_params(
                self.g, 0.7, self.h_dry, A.SWE_F64, self._q.size,
                self._q.ctypes.data_as(C.POINTER(C.c_double)),
                {"auto": A.SWE_AUTO, "cell": A.SWE_CELL, "tiled": A.SWE_TILED}[variant], 0)
            self._variant = variant
        return self.params

    def run_device(self, n, z, h, hu, hv, stream=None, variant="auto"):
        """J (a float; the call synchronises the stream) and its gradients (dn, dz, dh, dhu,
        dhv) as float64 tensors on the mesh's device in input order, from per-cell inputs in
        input order (tensors on that device are read in place; others are copied there)."""
        m = self.mesh
        t = m.n_cells
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            for k, a in enumerate((z, n, h, hu, hv)):
                a = torch.as_tensor(a)
                if a.shape != (t,):
                    raise ValueError(f"per-cell inputs must have shape ({t},), got {tuple(a.shape)}")
                a = a.to(device=m.device, dtype=torch.float64)   # no copy for device float64
                torch.index_select(a, 0, self.perm, out=self.fields[k])
            j = A.swe_adjoint(m.handle, m.dev, self._params(variant), self.state, self.n_steps,
                              _ptr(self.dt), self.loss, self.ckpt_every, self.grads,
                              _ptr(self.ws), self.ws.numel(), _stream_handle(stream))
            out = torch.empty((5, t), dtype=torch.float64, device=m.device)
            out.index_copy_(1, self.perm, self.grad_mesh)
        # in the order of swe_grads: dn, dz, dh, dhu, dhv
        return j, (out[0], out[1], out[2], out[3], out[4])

    def run(self, n, z, h, hu, hv, stream=None, variant="auto"):
        """J and its gradients (dn, dz, dh, dhu, dhv) as float64 numpy arrays in input order.
        variant: the step kernel of the forward passes ("tiled" also tiles the flux adjoint)."""
        d = self.mesh.device
        args = [torch.as_tensor(np.asarray(a, np.float64), device=d) for a in (n, z, h, hu, hv)]
        j, grads = self.run_device(*args, stream=stream, variant=variant)
        return j, tuple(g.cpu().numpy() for g in grads)


class AdjointLoss(torch.autograd.Function):
    """J(n, z, h0, hu0, hv0) of a Calibration; backward returns the adjoint's gradients, on the
    inputs' device, in their dtype."""

    @staticmethod
    def forward(ctx, calib: Calibration, n, z, h, hu, hv):
        j, grads = calib.run_device(*(t.detach() for t in (n, z, h, hu, hv)))
        ctx.grads = [g.to(device=t.device, dtype=t.dtype) for g, t in zip(grads, (n, z, h, hu, hv))]
        return torch.tensor(j, dtype=torch.float64, device=n.device)

    @staticmethod
    def backward(ctx, grad_out):
        return (None, *[g * grad_out.to(g.dtype) for g in ctx.grads])
