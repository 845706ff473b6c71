"""One mesh stepped as several shards: contiguous ranges of its (Morton) cell order, each with
its one-cell halo, as a run over several devices would lay it out.  Here all shards live on
one device: the halo exchange is swe_halo_pack on the owner, a device copy standing in for the
interconnect, and swe_halo_unpack on the receiver; the dt all-reduce is swe_shard_dt_combine.
Every step of every shard runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A
from .solver import Mesh, Solver, _cell_field, _ptr, _stream_handle


class ShardedSolver:
    """`parts` shards of `mesh`; fields are given in the mesh's input order, as for Solver."""

    def __init__(self, mesh: Mesh, parts: int, z, n, h, hu, hv, dtype: str = "f64",
                 bounds=None, **solver_kw):
        t = mesh.n_cells
        if bounds is None:
            bounds = np.linspace(0, t, parts + 1).round().astype(np.int64)
        self.bounds = np.asarray(bounds, np.int64)
        if self.bounds[0] != 0 or self.bounds[-1] != t or np.any(np.diff(self.bounds) <= 0):
            raise ValueError("shard bounds must rise strictly from 0 to n_cells")
        self.mesh = mesh
        self.parts = len(self.bounds) - 1
        dev = mesh.device
        full = [_cell_field(mesh, a, name) for a, name in zip((z, n, h, hu, hv),
                                                               ("z", "n", "h", "hu", "hv"))]
        self.meshes, self.solvers = [], []
        for p in range(self.parts):
            m = Mesh.shard(mesh, int(self.bounds[p]), int(self.bounds[p + 1]), device=dev)
            g = m.global_ids
            self.meshes.append(m)
            self.solvers.append(Solver(m, *[a[g] for a in full], dtype=dtype, shard=True,
                                       **solver_kw))
        self.dtype = self.solvers[0].dtype
        # exchange lists: the halo cells of shard q that shard p owns, in q's halo order
        self.links = []
        for q, m in enumerate(self.meshes):
            halo_g = m.global_ids[m.n_owned:].astype(np.int64)
            owner = np.searchsorted(self.bounds, halo_g, side="right") - 1
            for p in np.unique(owner):
                sel = np.flatnonzero(owner == p)
                send = torch.as_tensor((halo_g[sel] - self.bounds[p]).astype(np.int32), device=dev)
                recv = torch.as_tensor((m.n_owned + sel).astype(np.int32), device=dev)
                buf = torch.empty(3 * sel.size, dtype=self.solvers[q].tdtype, device=dev)
                self.links.append((int(p), q, send, recv, buf))
        self._ctrls = [s.ctrl.data_ptr() for s in self.solvers]
        self.exchange()
        self.combine()

    def exchange(self, stream=None) -> None:
        """Refresh every halo from its owner's current state."""
        st = _stream_handle(stream)
        for p, q, send, recv, buf in self.links:
            sp, sq = self.solvers[p], self.solvers[q]
            A.swe_halo_pack(self.dtype, send.numel(), _ptr(send), *[_ptr(x) for x in sp.device_state()],
                            _ptr(buf), st)
            A.swe_halo_unpack(self.dtype, recv.numel(), _ptr(recv), _ptr(buf),
                              *[_ptr(x) for x in sq.device_state()], st)

    def combine(self, stream=None) -> None:
        """The dt all-reduce: every shard's next dt becomes the minimum of their candidates."""
        A.swe_shard_dt_combine(self._ctrls, _stream_handle(stream))

    def step(self, n_steps: int = 1, stream=None) -> None:
        for _ in range(n_steps):
            for s in self.solvers:
                s.step(stream)
            self.exchange(stream)
            self.combine(stream)

    def stats(self, stream=None):
        """(status, stats) of the sharded run: time and steps of shard 0 (all shards agree),
        clamps summed over shards."""
        res = [s.stats(stream) for s in self.solvers]
        rc = next((r for r, _ in res if r != A.SWE_OK), A.SWE_OK)
        st = dict(res[0][1])
        st["clamps"] = sum(x["clamps"] for _, x in res)
        return rc, st

    def numpy_state(self):
        """The owned cells of every shard, assembled in the mesh's input order."""
        t = self.mesh.n_cells
        out = [np.empty(t), np.empty(t), np.empty(t)]
        for m, s in zip(self.meshes, self.solvers):
            s.stats()
            g = m.global_ids[:m.n_owned]
            for o, x in zip(out, s.device_state()):
                o[g] = x[:m.n_owned].double().cpu().numpy()
        return tuple(self.mesh.to_input_order(o) for o in out)
