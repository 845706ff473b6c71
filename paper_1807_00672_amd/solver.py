"""Mesh and Solver: torch-owned device memory around the libswe C ABI.

torch provides device memory and the stream; the library's kernels do all the work.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _cell_field(mesh, a, name: str) -> np.ndarray:
    """A per-cell input (one value per cell, input order) as float64 in mesh order; the kernels
    index it by cell, so any other shape is refused here."""
    a = np.asarray(a, np.float64)
    if a.shape != (mesh.n_cells,):
        raise ValueError(f"{name} must hold one value per cell: shape ({mesh.n_cells},), "
                         f"got {a.shape}")
    return mesh.to_mesh_order(a)


def _tuned_tile(n_cells: int, dtype: str) -> int:
    """The tile size swe_tune's table holds for this device, precision and size class."""
    dev = torch.cuda.current_device() if torch.cuda.is_available() else 0
    r = A.swe_tune_get(dev, {"f64": A.SWE_F64, "f32": A.SWE_F32}[dtype], n_cells)
    return int(r.tile_cells) if r.variant != A.SWE_AUTO and r.tile_cells in A.TILE_FLAGS else A.SWE_TILE


class Mesh:
    """A triangle mesh built by swe_mesh_create, with its arrays copied to the device.

    xy: [V, 2] node coordinates; tri: [T, 3] node ids (either orientation); edge_tag: optional
    [T, 3] boundary tags (0 wall, s >= 1 inflow segment s) of input edge (k, k+1).
    """

    ORDERS = {"morton": A.SWE_MORTON, "hilbert": A.SWE_HILBERT, "input": 0}

    def __init__(self, xy, tri, edge_tag=None, morton: bool = True, device="cuda", handle=None,
                 order: str | None = None, tile: int | str = A.SWE_TILE, dtype: str = "f64"):
        """order: "morton", "hilbert" or "input" cell order (default: morton unless morton=False).
        tile: cells per tile (64, 128, 256 or 512), or "auto": the size swe_tune recorded as
        fastest for this device, `dtype` and size class (tune.tune_tiles), else SWE_TILE."""
        flags = self.ORDERS[order or ("morton" if morton else "input")]
        if tile == "auto":
            tile = _tuned_tile(len(tri), dtype)
        if tile not in A.TILE_FLAGS:
            raise ValueError(f"tile must be 64, 128, 256 or 512, not {tile!r}")
        flags |= A.TILE_FLAGS[tile]
        self.handle = handle if handle is not None else A.swe_mesh_create(xy, tri, edge_tag, flags)
        self.info = A.swe_mesh_info_get(self.handle)
        t, v = int(self.info.n_cells), int(self.info.n_nodes)
        self.n_cells, self.n_nodes = t, v
        self.tile = int(self.info.tile_cells)
        self.perm = A.swe_mesh_export(self.handle, A.SWE_ARR_PERM, t, np.int32)
        self.nbr = A.swe_mesh_export(self.handle, A.SWE_ARR_NBR, 3 * t, np.int32)
        self.c2n = A.swe_mesh_export(self.handle, A.SWE_ARR_C2N, 3 * t, np.int32)
        self.xy = A.swe_mesh_export(self.handle, A.SWE_ARR_XY, 2 * v, np.float64)
        self.node_perm = A.swe_mesh_export(self.handle, A.SWE_ARR_NODE_PERM, v, np.int32)
        nt = int(self.info.n_tiles)
        self.halo_off = A.swe_mesh_export(self.handle, A.SWE_ARR_HALO_OFF, nt + 1, np.int32)
        self.halo = A.swe_mesh_export(self.handle, A.SWE_ARR_HALO, max(1, int(self.info.n_halo)),
                                      np.int32)
        self.edge_off = A.swe_mesh_export(self.handle, A.SWE_ARR_EDGE_OFF, nt + 1, np.int32)
        self.edges = A.swe_mesh_export(self.handle, A.SWE_ARR_EDGES, int(self.info.n_tile_edges),
                                       np.uint32)
        self.slot = A.swe_mesh_export(self.handle, A.SWE_ARR_SLOT, 3 * t, np.uint16)
        self.edge_vec = A.swe_mesh_export(self.handle, A.SWE_ARR_EDGE_VEC,
                                          2 * int(self.info.n_tile_edges), np.float64)
        self.cell_geo = A.swe_mesh_export(self.handle, A.SWE_ARR_CELL_GEO, 2 * t, np.float64)
        self.edge_vec32 = A.swe_mesh_export(self.handle, A.SWE_ARR_EDGE_VEC32,
                                            2 * int(self.info.n_tile_edges), np.float32)
        self.cell_geo32 = A.swe_mesh_export(self.handle, A.SWE_ARR_CELL_GEO32, 2 * t, np.float32)
        # tile node lists (none where a tile has more than 256 nodes)
        self.tile_node_off = self.tile_nodes = self.edge_nodes = None
        if int(self.info.n_tile_nodes) > 0:
            self.tile_node_off = A.swe_mesh_export(self.handle, A.SWE_ARR_TILE_NODE_OFF, nt + 1,
                                                   np.int32)
            self.tile_nodes = A.swe_mesh_export(self.handle, A.SWE_ARR_TILE_NODES,
                                                2 * int(self.info.n_tile_nodes), np.float64)
            self.edge_nodes = A.swe_mesh_export(self.handle, A.SWE_ARR_EDGE_NODES,
                                                int(self.info.n_tile_edges), np.uint16)
        self.n_owned = int(self.info.n_owned)
        self.global_ids = A.swe_mesh_export(self.handle, A.SWE_ARR_GLOBAL, t, np.int32)
        self.device = None
        if device is not None:
            self.to(device)

    @classmethod
    def shard(cls, full: "Mesh", c0: int, c1: int, device="cuda") -> "Mesh":
        """Cells [c0, c1) of `full` (its mesh order) followed by their halo, as a mesh of its own
        (swe_mesh_create_shard); `global_ids` maps its cells to `full`'s."""
        return cls(None, None, handle=A.swe_mesh_create_shard(full.handle, c0, c1), device=device)

    def to(self, device="cuda"):
        d = torch.device(device)
        if d.type == "cuda" and d.index is None:
            d = torch.device("cuda", torch.cuda.current_device())
        self.device = d
        self.d_nbr = torch.from_numpy(self.nbr).to(self.device)
        self.d_c2n = torch.from_numpy(self.c2n).to(self.device)
        self.d_xy = torch.from_numpy(self.xy).to(self.device)
        self.d_halo_off = torch.from_numpy(self.halo_off).to(self.device)
        self.d_halo = torch.from_numpy(self.halo).to(self.device)
        self.d_edge_off = torch.from_numpy(self.edge_off).to(self.device)
        self.d_edges = torch.from_numpy(self.edges.view(np.int32)).to(self.device)
        self.d_slot = torch.from_numpy(self.slot.view(np.int16)).to(self.device)
        self.d_edge_vec = torch.from_numpy(self.edge_vec).to(self.device)
        self.d_cell_geo = torch.from_numpy(self.cell_geo).to(self.device)
        self.d_edge_vec32 = torch.from_numpy(self.edge_vec32).to(self.device)
        self.d_cell_geo32 = torch.from_numpy(self.cell_geo32).to(self.device)
        nodes = self.tile_nodes is not None
        self.d_tile_node_off = torch.from_numpy(self.tile_node_off).to(self.device) if nodes else None
        self.d_tile_nodes = torch.from_numpy(self.tile_nodes).to(self.device) if nodes else None
        self.d_edge_nodes = (torch.from_numpy(self.edge_nodes.view(np.int16)).to(self.device)
                             if nodes else None)
        opt = lambda t: _ptr(t) if t is not None else None
        self.dev = A.swe_dev_mesh(self.n_cells, self.n_nodes, _ptr(self.d_nbr), _ptr(self.d_c2n),
                                  _ptr(self.d_xy), _ptr(self.d_halo_off), _ptr(self.d_halo),
                                  _ptr(self.d_edge_off), _ptr(self.d_edges), _ptr(self.d_slot),
                                  _ptr(self.d_edge_vec), _ptr(self.d_cell_geo),
                                  _ptr(self.d_edge_vec32), _ptr(self.d_cell_geo32),
                                  opt(self.d_tile_node_off), opt(self.d_tile_nodes),
                                  opt(self.d_edge_nodes))
        return self

    def to_mesh_order(self, a):
        return np.asarray(a)[self.perm]

    def to_input_order(self, a):
        a = np.asarray(a)
        out = np.empty_like(a)
        out[self.perm] = a
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and A is not None and A.lib is not None:
            A.swe_mesh_destroy(h)
            self.handle = None


class Solver:
    """One simulation state on the device: U = (h, hu, hv) ping-pong buffers, bed, roughness,
    the control block (time, dt, counters) and the reduction workspace."""

    VARIANTS = {"auto": A.SWE_AUTO, "cell": A.SWE_CELL, "tiled": A.SWE_TILED}

    def __init__(self, mesh: Mesh, z, n, h, hu, hv, dtype: str = "f64", g=9.81, courant=0.7,
                 h_dry=1e-6, inflow_q=None, t0=0.0, t_end=0.0, stream=None, variant="auto",
                 xcd_remap=True, shard=False, index64=False, exact=False):
        if mesh.device is None:
            raise ValueError("mesh has no device arrays")
        self.mesh = mesh
        self.dtype = {"f64": A.SWE_F64, "f32": A.SWE_F32}[dtype]
        self.tdtype = torch.float64 if self.dtype == A.SWE_F64 else torch.float32
        dev = mesh.device
        self._q = np.ascontiguousarray(inflow_q if inflow_q is not None else [], np.float64)
        self.params = A.swe_params(g, courant, h_dry, self.dtype, self._q.size,
                                   self._q.ctypes.data_as(C.POINTER(C.c_double)),
                                   self.VARIANTS[variant],
                                   (0 if xcd_remap else A.SWE_NO_XCD_REMAP) |
                                   (A.SWE_SHARD if shard else 0) |
                                   (A.SWE_INDEX64 if index64 else 0) |
                                   (A.SWE_EXACT if exact else 0))
        t = mesh.n_cells

        def field(a, name):
            return torch.from_numpy(_cell_field(mesh, a, name)).to(
                device=dev, dtype=self.tdtype).contiguous()

        self.z, self.n = field(z, "z"), field(n, "n")
        self.h = [field(h, "h"), torch.empty(t, dtype=self.tdtype, device=dev)]
        self.hu = [field(hu, "hu"), torch.empty(t, dtype=self.tdtype, device=dev)]
        self.hv = [field(hv, "hv"), torch.empty(t, dtype=self.tdtype, device=dev)]
        self.ctrl = torch.zeros(A.SWE_CTRL_BYTES // 8, dtype=torch.float64, device=dev)
        self.work = torch.zeros(A.swe_workspace_bytes(t), dtype=torch.uint8, device=dev)
        self.state = A.swe_state(
            (C.c_void_p * 2)(self.h[0].data_ptr(), self.h[1].data_ptr()),
            (C.c_void_p * 2)(self.hu[0].data_ptr(), self.hu[1].data_ptr()),
            (C.c_void_p * 2)(self.hv[0].data_ptr(), self.hv[1].data_ptr()),
            _ptr(self.z), _ptr(self.n), _ptr(self.ctrl), _ptr(self.work), 0, 0)
        self.init(t0, t_end, stream)

    def init(self, t0=0.0, t_end=0.0, stream=None):
        A.swe_state_init(self.mesh.handle, self.mesh.dev, self.params, self.state, t0, t_end,
                         _stream_handle(stream))

    def step(self, stream=None):
        A.swe_step(self.mesh.handle, self.mesh.dev, self.params, self.state, _stream_handle(stream))

    def run(self, n_steps: int, dt_seq: torch.Tensor | None = None, sync: bool = True,
            stream=None):
        """Queue n_steps steps; with sync, wait and return (status code, stats dict)."""
        seq = None
        if dt_seq is not None:
            if dt_seq.dtype != torch.float64 or dt_seq.device != self.mesh.device:
                raise ValueError("dt_seq must be a float64 tensor on the mesh device")
            if dt_seq.numel() < n_steps:
                raise ValueError(f"dt_seq holds {dt_seq.numel()} values for {n_steps} steps")
            self._dt_seq = dt_seq.contiguous()   # alive while the queued steps read it
            seq = _ptr(self._dt_seq)
        st = A.swe_run_stats() if sync else None
        rc = A.swe_run(self.mesh.handle, self.mesh.dev, self.params, self.state, n_steps, seq,
                       st, _stream_handle(stream))
        return (rc, st.as_dict()) if sync else None

    def stats(self, stream=None):
        st = A.swe_run_stats()
        rc = A.swe_read_stats(self.state, st, _stream_handle(stream))
        return rc, st.as_dict()

    @property
    def cur(self) -> int:
        return int(self.state.cur)

    def device_state(self):
        """The current (h, hu, hv) device tensors, mesh order."""
        c = self.cur
        return self.h[c], self.hu[c], self.hv[c]

    def numpy_state(self):
        """The current state as float64 numpy arrays in input order (synchronises)."""
        self.stats()
        return tuple(self.mesh.to_input_order(t.double().cpu().numpy())
                     for t in self.device_state())


class Batch:
    """Several meshes (scenarios) concatenated by swe_batch_create, with device arrays."""

    def __init__(self, meshes, device="cuda"):
        self.meshes = list(meshes)
        self.handle = A.swe_batch_create([m.handle for m in self.meshes])
        self.info = A.swe_batch_info_get(self.handle)
        i = self.info
        n, t, v, nt = int(i.n_scenarios), int(i.n_cells), int(i.n_nodes), int(i.n_tiles)
        self.n_scen, self.n_cells, self.n_nodes = n, t, v
        ex = lambda w, k, dt: A.swe_batch_export(self.handle, w, k, dt)
        self.cell_off = ex(A.SWE_BARR_CELL_OFF, n + 1, np.int64)
        arrays = {
            "nbr": ex(A.SWE_ARR_NBR, 3 * t, np.int32), "c2n": ex(A.SWE_ARR_C2N, 3 * t, np.int32),
            "xy": ex(A.SWE_ARR_XY, 2 * v, np.float64),
            "halo_off": ex(A.SWE_ARR_HALO_OFF, nt + 1, np.int32),
            "halo": ex(A.SWE_ARR_HALO, max(1, int(i.n_halo)), np.int32),
            "edge_off": ex(A.SWE_ARR_EDGE_OFF, nt + 1, np.int32),
            "edges": ex(A.SWE_ARR_EDGES, int(i.n_tile_edges), np.uint32).view(np.int32),
            "slot": ex(A.SWE_ARR_SLOT, 3 * t, np.uint16).view(np.int16),
            "edge_vec": ex(A.SWE_ARR_EDGE_VEC, 2 * int(i.n_tile_edges), np.float64),
            "cell_geo": ex(A.SWE_ARR_CELL_GEO, 2 * t, np.float64),
            "edge_vec32": ex(A.SWE_ARR_EDGE_VEC32, 2 * int(i.n_tile_edges), np.float32),
            "cell_geo32": ex(A.SWE_ARR_CELL_GEO32, 2 * t, np.float32),
            "tile_start": ex(A.SWE_BARR_TILE_START, nt + 1, np.int32),
            "tile_scen": ex(A.SWE_BARR_TILE_SCEN, nt, np.int32),
            "scen_tile_off": ex(A.SWE_BARR_SCEN_TILE_OFF, n + 1, np.int32),
        }
        if int(i.n_tile_nodes) > 0:   # every scenario has tile node lists
            arrays["tile_node_off"] = ex(A.SWE_ARR_TILE_NODE_OFF, nt + 1, np.int32)
            arrays["tile_nodes"] = ex(A.SWE_ARR_TILE_NODES, 2 * int(i.n_tile_nodes), np.float64)
            arrays["edge_nodes"] = ex(A.SWE_ARR_EDGE_NODES, int(i.n_tile_edges),
                                      np.uint16).view(np.int16)
        d = torch.device(device)
        if d.type == "cuda" and d.index is None:
            d = torch.device("cuda", torch.cuda.current_device())
        self.device = d
        self.d = {k: torch.from_numpy(a).to(d) for k, a in arrays.items()}
        P = lambda k: _ptr(self.d[k]) if k in self.d else None
        mesh = A.swe_dev_mesh(t, v, P("nbr"), P("c2n"), P("xy"), P("halo_off"), P("halo"),
                              P("edge_off"), P("edges"), P("slot"), P("edge_vec"), P("cell_geo"),
                              P("edge_vec32"), P("cell_geo32"), P("tile_node_off"),
                              P("tile_nodes"), P("edge_nodes"))
        self.dev = A.swe_batch_dev(mesh, P("tile_start"), P("tile_scen"), P("scen_tile_off"))

    def scenario_slice(self, s: int) -> slice:
        return slice(int(self.cell_off[s]), int(self.cell_off[s + 1]))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and A is not None and A.lib is not None:
            A.swe_batch_destroy(h)
            self.handle = None


class BatchSolver:
    """All scenarios' states in concatenated buffers; one launch per step steps them all."""

    def __init__(self, batch: Batch, cases, dtype="f64", g=9.81, courant=0.7, h_dry=1e-6,
                 t0=0.0, t_end=0.0, stream=None, variant="auto", xcd_remap=True, exact=False):
        self.batch = batch
        self.tdtype = torch.float64 if dtype == "f64" else torch.float32
        dev = batch.device
        cases = list(cases)
        if len(cases) != batch.n_scen:
            raise ValueError(f"need one case per scenario: {batch.n_scen}, got {len(cases)}")
        q = np.zeros((batch.n_scen, A.SWE_MAX_INFLOW))
        cat = {k: [] for k in ("z", "n", "h", "hu", "hv")}
        for s, (m, c) in enumerate(zip(batch.meshes, cases)):
            for k in cat:
                cat[k].append(_cell_field(m, getattr(c, k), f"scenario {s} {k}"))
            if c.inflow_q is not None:
                q[s, : len(c.inflow_q)] = c.inflow_q
        f = {k: torch.from_numpy(np.concatenate(v)).to(device=dev, dtype=self.tdtype)
             for k, v in cat.items()}
        t = batch.n_cells
        self.z, self.n = f["z"], f["n"]
        self.h = [f["h"], torch.empty(t, dtype=self.tdtype, device=dev)]
        self.hu = [f["hu"], torch.empty(t, dtype=self.tdtype, device=dev)]
        self.hv = [f["hv"], torch.empty(t, dtype=self.tdtype, device=dev)]
        self.q = torch.from_numpy(q.ravel()).to(dev)
        self.ctrl = torch.zeros(batch.n_scen * A.SWE_CTRL_BYTES // 8, dtype=torch.float64,
                                device=dev)
        self.work = torch.zeros(A.swe_batch_workspace_bytes(batch.handle), dtype=torch.uint8,
                                device=dev)
        self.params = A.swe_batch_params(g, courant, h_dry,
                                         A.SWE_F64 if dtype == "f64" else A.SWE_F32,
                                         Solver.VARIANTS[variant], _ptr(self.q),
                                         (0 if xcd_remap else A.SWE_NO_XCD_REMAP) |
                                         (A.SWE_EXACT if exact else 0), 0)
        self.state = A.swe_state(
            (C.c_void_p * 2)(self.h[0].data_ptr(), self.h[1].data_ptr()),
            (C.c_void_p * 2)(self.hu[0].data_ptr(), self.hu[1].data_ptr()),
            (C.c_void_p * 2)(self.hv[0].data_ptr(), self.hv[1].data_ptr()),
            _ptr(self.z), _ptr(self.n), _ptr(self.ctrl), _ptr(self.work), 0, 0)
        A.swe_batch_state_init(batch.handle, batch.dev, self.params, self.state, t0, t_end,
                               _stream_handle(stream))
        self.last = None

    def run(self, n_steps: int, sync=True, stream=None):
        st = (A.swe_run_stats * self.batch.n_scen)() if sync else None
        rc = A.swe_batch_run(self.batch.handle, self.batch.dev, self.params, self.state, n_steps,
                             st, _stream_handle(stream))
        if sync:
            self.last = [x.as_dict() for x in st]
            return rc, self.last
        return None

    def numpy_state(self, s: int):
        """Scenario s's (h, hu, hv) in its input order (after a synchronising run)."""
        if self.last is None:
            self.run(0)
        c = self.last[s]["cur"]
        sl = self.batch.scenario_slice(s)
        m = self.batch.meshes[s]
        return tuple(m.to_input_order(b[c][sl].double().cpu().numpy())
                     for b in (self.h, self.hu, self.hv))
