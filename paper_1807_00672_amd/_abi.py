"""ctypes binding of libswe.so with the C ABI's names (include/swe.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the library.
A missing or unloadable library raises at import; there is no other implementation to fall
back to.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library then shares)

HERE = os.path.dirname(os.path.abspath(__file__))
# SWE_LIB may name another build of the same sources (kernel-tuning builds); default in-tree.
LIB_PATH = os.environ.get("SWE_LIB") or os.path.join(HERE, "libswe.so")

SWE_OK = 0
SWE_EINVAL = -1
SWE_EMESH = -2
SWE_EDEVICE = -3
SWE_ENONFINITE = -4
SWE_EDRY = -5
SWE_EUNSUPPORTED = -6

SWE_F64 = 0
SWE_F32 = 1
SWE_MORTON = 1
SWE_HILBERT = 2
SWE_MAX_INFLOW = 16
SWE_CTRL_BYTES = 512
SWE_WALL = -1

SWE_AUTO, SWE_CELL, SWE_TILED = 0, 1, 2
SWE_NO_XCD_REMAP = 1
SWE_SHARD = 2
SWE_INDEX64 = 4
SWE_EXACT = 8
SWE_TILE = 256
SWE_TILE_64, SWE_TILE_128, SWE_TILE_512 = 16, 32, 64
TILE_FLAGS = {64: SWE_TILE_64, 128: SWE_TILE_128, 256: 0, 512: SWE_TILE_512}
# packed edge-list entry: side a, a's local edge, b's local edge, side b (int16)
EDGE_A_MASK, EDGE_KA_SHIFT, EDGE_KB_SHIFT = 0x1FF, 9, 11

(SWE_ARR_PERM, SWE_ARR_NBR, SWE_ARR_C2N, SWE_ARR_XY, SWE_ARR_NODE_PERM, SWE_ARR_HALO_OFF,
 SWE_ARR_HALO, SWE_ARR_EDGE_OFF, SWE_ARR_EDGES, SWE_ARR_SLOT, SWE_ARR_GLOBAL, SWE_ARR_EDGE_VEC,
 SWE_ARR_CELL_GEO, SWE_ARR_EDGE_VEC32, SWE_ARR_CELL_GEO32) = range(15)
SWE_ARR_TILE_NODE_OFF, SWE_ARR_TILE_NODES, SWE_ARR_EDGE_NODES = 21, 22, 23

_NAMES = {0: "SWE_OK", -1: "SWE_EINVAL", -2: "SWE_EMESH", -3: "SWE_EDEVICE",
          -4: "SWE_ENONFINITE", -5: "SWE_EDRY", -6: "SWE_EUNSUPPORTED"}


class SweError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class swe_mesh_info(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_nodes", C.c_int64), ("n_edges", C.c_int64),
                ("n_boundary_edges", C.c_int64), ("n_inflow_edges", C.c_int64),
                ("n_inflow_segments", C.c_int32), ("flags", C.c_uint32),
                ("min_area", C.c_double), ("max_area", C.c_double),
                ("total_area", C.c_double), ("min_inradius", C.c_double),
                ("bbox", C.c_double * 4), ("n_tiles", C.c_int64), ("n_halo", C.c_int64),
                ("n_tile_edges", C.c_int64), ("max_halo", C.c_int32),
                ("max_tile_edges", C.c_int32), ("n_owned", C.c_int64),
                ("n_tile_nodes", C.c_int64), ("max_tile_nodes", C.c_int32),
                ("tile_cells", C.c_int32)]


class swe_dev_mesh(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_nodes", C.c_int64), ("nbr", C.c_void_p),
                ("c2n", C.c_void_p), ("xy", C.c_void_p), ("halo_off", C.c_void_p),
                ("halo", C.c_void_p), ("edge_off", C.c_void_p), ("edges", C.c_void_p),
                ("slot", C.c_void_p), ("edge_vec", C.c_void_p), ("cell_geo", C.c_void_p),
                ("edge_vec32", C.c_void_p), ("cell_geo32", C.c_void_p),
                ("tile_node_off", C.c_void_p), ("tile_nodes", C.c_void_p),
                ("edge_nodes", C.c_void_p)]


class swe_params(C.Structure):
    _fields_ = [("g", C.c_double), ("courant", C.c_double), ("h_dry", C.c_double),
                ("dtype", C.c_int32), ("n_inflow", C.c_int32),
                ("inflow_q", C.POINTER(C.c_double)), ("variant", C.c_int32),
                ("flags", C.c_int32)]


class swe_state(C.Structure):
    _fields_ = [("h", C.c_void_p * 2), ("hu", C.c_void_p * 2), ("hv", C.c_void_p * 2),
                ("z", C.c_void_p), ("n", C.c_void_p), ("ctrl", C.c_void_p), ("work", C.c_void_p),
                ("cur", C.c_int32), ("reserved", C.c_int32)]


class swe_run_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("clamps", C.c_int64), ("t", C.c_double),
                ("dt_next", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double),
                ("dt_sum", C.c_double), ("status", C.c_int32), ("done", C.c_int32),
                ("cur", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


SWE_BARR_CELL_OFF, SWE_BARR_NODE_OFF, SWE_BARR_TILE_START, SWE_BARR_TILE_SCEN, \
    SWE_BARR_SCEN_TILE_OFF = range(16, 21)


class swe_tune_result(C.Structure):
    _fields_ = [("variant", C.c_int32), ("xcd_remap", C.c_int32),
                ("ms_per_step", C.c_double * 4), ("tile_cells", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return {"variant": {SWE_AUTO: "auto", SWE_CELL: "cell", SWE_TILED: "tiled"}[self.variant],
                "xcd_remap": bool(self.xcd_remap), "tile": int(self.tile_cells),
                "ms_per_step": {k: self.ms_per_step[i] for i, k in
                                enumerate(("cell+remap", "cell", "tiled+remap", "tiled"))}}

class swe_batch_info(C.Structure):
    _fields_ = [("n_scenarios", C.c_int32), ("max_inflow_segments", C.c_int32),
                ("n_cells", C.c_int64), ("n_nodes", C.c_int64), ("n_tiles", C.c_int64),
                ("n_halo", C.c_int64), ("n_tile_edges", C.c_int64), ("max_halo", C.c_int32),
                ("max_tile_edges", C.c_int32), ("n_tile_nodes", C.c_int64),
                ("max_tile_nodes", C.c_int32), ("tile_cells", C.c_int32)]


class swe_batch_dev(C.Structure):
    _fields_ = [("mesh", swe_dev_mesh), ("tile_start", C.c_void_p), ("tile_scen", C.c_void_p),
                ("scen_tile_off", C.c_void_p)]


class swe_batch_params(C.Structure):
    _fields_ = [("g", C.c_double), ("courant", C.c_double), ("h_dry", C.c_double),
                ("dtype", C.c_int32), ("variant", C.c_int32), ("inflow_q", C.c_void_p),
                ("flags", C.c_int32), ("reserved", C.c_int32)]


class swe_loss(C.Structure):
    _fields_ = [("gauges", C.c_void_p), ("n_gauges", C.c_int32), ("every", C.c_int32),
                ("obs", C.c_void_p)]


class swe_grads(C.Structure):
    _fields_ = [("dn", C.c_void_p), ("dz", C.c_void_p), ("dh", C.c_void_p), ("dhu", C.c_void_p),
                ("dhv", C.c_void_p)]


EXPORTS = [
    "swe_mesh_create", "swe_mesh_info_get", "swe_mesh_export", "swe_mesh_destroy",
    "swe_workspace_bytes", "swe_state_init", "swe_step", "swe_run", "swe_read_stats",
    "swe_last_error", "swe_flux_eval", "swe_batch_create", "swe_batch_info_get",
    "swe_batch_export", "swe_batch_destroy", "swe_batch_workspace_bytes", "swe_batch_state_init",
    "swe_batch_run", "swe_adjoint_workspace_bytes", "swe_adjoint", "swe_adjoint_timings", "swe_tune", "swe_tune_get",
    "swe_tune_set", "swe_mesh_create_shard", "swe_halo_pack", "swe_halo_unpack",
    "swe_shard_dt_combine", "swe_run_static",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(hipcc for gfx950); there is no fallback implementation")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.swe_mesh_create.argtypes = [vp, i64, vp, i64, vp, C.c_uint32, C.POINTER(vp)]
    L.swe_mesh_info_get.argtypes = [vp, C.POINTER(swe_mesh_info)]
    L.swe_mesh_export.argtypes = [vp, i32, vp, i64]
    L.swe_mesh_destroy.argtypes = [vp]
    L.swe_mesh_destroy.restype = None
    L.swe_workspace_bytes.argtypes = [i64, C.POINTER(i64)]
    L.swe_state_init.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                                 C.POINTER(swe_state), dbl, dbl, vp]
    L.swe_step.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                           C.POINTER(swe_state), vp]
    L.swe_run.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                          C.POINTER(swe_state), i64, vp, C.POINTER(swe_run_stats), vp]
    L.swe_read_stats.argtypes = [C.POINTER(swe_state), C.POINTER(swe_run_stats), vp]
    L.swe_run_static.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                                 C.POINTER(swe_state), i32, dbl, dbl, i64, vp,
                                 C.POINTER(swe_run_stats), vp]
    L.swe_last_error.argtypes = []
    L.swe_last_error.restype = C.c_char_p
    L.swe_flux_eval.argtypes = [i32, i32, i64, dbl, dbl] + [vp] * 12 + [vp]
    L.swe_adjoint_timings.argtypes = [C.POINTER(dbl), C.POINTER(dbl)]
    L.swe_mesh_create_shard.argtypes = [vp, i64, i64, C.POINTER(vp)]
    L.swe_halo_pack.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    L.swe_halo_unpack.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    L.swe_shard_dt_combine.argtypes = [C.POINTER(vp), i32, vp]
    L.swe_tune.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                           C.POINTER(swe_state), i32, C.POINTER(swe_tune_result), vp]
    L.swe_tune_get.argtypes = [i32, i32, i64, C.POINTER(swe_tune_result)]
    L.swe_tune_set.argtypes = [i32, i32, i64, C.POINTER(swe_tune_result)]
    L.swe_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    L.swe_batch_info_get.argtypes = [vp, C.POINTER(swe_batch_info)]
    L.swe_batch_export.argtypes = [vp, i32, vp, i64]
    L.swe_batch_destroy.argtypes = [vp]
    L.swe_batch_destroy.restype = None
    L.swe_batch_workspace_bytes.argtypes = [vp, C.POINTER(i64)]
    L.swe_batch_state_init.argtypes = [vp, C.POINTER(swe_batch_dev), C.POINTER(swe_batch_params),
                                       C.POINTER(swe_state), dbl, dbl, vp]
    L.swe_batch_run.argtypes = [vp, C.POINTER(swe_batch_dev), C.POINTER(swe_batch_params),
                                C.POINTER(swe_state), i64, vp, vp]
    L.swe_adjoint_workspace_bytes.argtypes = [vp, i64, i32, C.POINTER(i64)]
    L.swe_adjoint.argtypes = [vp, C.POINTER(swe_dev_mesh), C.POINTER(swe_params),
                              C.POINTER(swe_state), i64, vp, C.POINTER(swe_loss), i32,
                              C.POINTER(swe_grads), C.POINTER(dbl), vp, i64, vp]
    for name in EXPORTS:
        if name not in ("swe_mesh_destroy", "swe_last_error", "swe_batch_destroy"):
            getattr(L, name).restype = i32
    return L


lib = _load()


def swe_last_error() -> str:
    return lib.swe_last_error().decode()


def _check(rc: int, where: str) -> int:
    if rc != SWE_OK:
        raise SweError(rc, where, swe_last_error())
    return rc


def _np_ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def swe_mesh_create(xy, tri, edge_tag=None, flags: int = SWE_MORTON) -> C.c_void_p:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    tag = None if edge_tag is None else np.ascontiguousarray(edge_tag, np.int32).reshape(-1, 3)
    out = C.c_void_p()
    _check(lib.swe_mesh_create(_np_ptr(xy), xy.shape[0], _np_ptr(tri), tri.shape[0],
                               None if tag is None else _np_ptr(tag), flags, C.byref(out)),
           "swe_mesh_create")
    return out


def swe_mesh_info_get(mesh) -> swe_mesh_info:
    info = swe_mesh_info()
    _check(lib.swe_mesh_info_get(mesh, C.byref(info)), "swe_mesh_info_get")
    return info


def swe_mesh_export(mesh, which: int, n: int, dtype) -> np.ndarray:
    out = np.empty(n, dtype=dtype)
    _check(lib.swe_mesh_export(mesh, which, _np_ptr(out), out.nbytes), "swe_mesh_export")
    return out


def swe_mesh_destroy(mesh) -> None:
    lib.swe_mesh_destroy(mesh)


def swe_workspace_bytes(n_cells: int) -> int:
    b = C.c_int64()
    _check(lib.swe_workspace_bytes(n_cells, C.byref(b)), "swe_workspace_bytes")
    return int(b.value)


def swe_state_init(mesh, dm, params, state, t0=0.0, t_end=0.0, stream=None) -> None:
    _check(lib.swe_state_init(mesh, C.byref(dm), C.byref(params), C.byref(state), t0, t_end,
                              stream), "swe_state_init")


def swe_step(mesh, dm, params, state, stream=None) -> None:
    _check(lib.swe_step(mesh, C.byref(dm), C.byref(params), C.byref(state), stream), "swe_step")


def swe_run(mesh, dm, params, state, n_steps: int, dt_seq=None, stats=None, stream=None) -> int:
    """Queue n_steps steps; with a stats record, synchronise and return the state's status."""
    rc = lib.swe_run(mesh, C.byref(dm), C.byref(params), C.byref(state), n_steps, dt_seq,
                     None if stats is None else C.byref(stats), stream)
    if rc in (SWE_EINVAL, SWE_EDEVICE, SWE_EMESH, SWE_EUNSUPPORTED):
        _check(rc, "swe_run")
    return rc


def swe_run_static(mesh, dm, params, state, n_steps: int, init: bool = False, t0=0.0,
                   t_end=0.0, dt_seq=None, stats=None, stream=None) -> int:
    """swe_state_init (init) and swe_run without a workspace; as swe_run otherwise."""
    rc = lib.swe_run_static(mesh, C.byref(dm), C.byref(params), C.byref(state), 1 if init else 0,
                            t0, t_end, n_steps, dt_seq, None if stats is None else C.byref(stats),
                            stream)
    if rc in (SWE_EINVAL, SWE_EDEVICE, SWE_EMESH, SWE_EUNSUPPORTED):
        _check(rc, "swe_run_static")
    return rc


def swe_read_stats(state, stats, stream=None) -> int:
    rc = lib.swe_read_stats(C.byref(state), C.byref(stats), stream)
    if rc in (SWE_EINVAL, SWE_EDEVICE):
        _check(rc, "swe_read_stats")
    return rc


def swe_flux_eval(dtype, n, g, h_dry, hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny, f, p,
                  stream=None, flags=0) -> None:
    _check(lib.swe_flux_eval(dtype, flags, n, g, h_dry, hl, hul, hvl, zl, hr, hur, hvr, zr, nx,
                             ny, f, p, stream), "swe_flux_eval")


def swe_batch_create(meshes) -> C.c_void_p:
    arr = (C.c_void_p * len(meshes))(*[m.value if isinstance(m, C.c_void_p) else m for m in meshes])
    out = C.c_void_p()
    _check(lib.swe_batch_create(arr, len(meshes), C.byref(out)), "swe_batch_create")
    return out


def swe_batch_info_get(batch) -> swe_batch_info:
    info = swe_batch_info()
    _check(lib.swe_batch_info_get(batch, C.byref(info)), "swe_batch_info_get")
    return info


def swe_batch_export(batch, which: int, n: int, dtype) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=dtype)
    _check(lib.swe_batch_export(batch, which, _np_ptr(out), out.nbytes), "swe_batch_export")
    return out[:n]


def swe_batch_destroy(batch) -> None:
    lib.swe_batch_destroy(batch)


def swe_batch_workspace_bytes(batch) -> int:
    b = C.c_int64()
    _check(lib.swe_batch_workspace_bytes(batch, C.byref(b)), "swe_batch_workspace_bytes")
    return int(b.value)


def swe_batch_state_init(batch, dev, params, state, t0=0.0, t_end=0.0, stream=None) -> None:
    _check(lib.swe_batch_state_init(batch, C.byref(dev), C.byref(params), C.byref(state), t0,
                                    t_end, stream), "swe_batch_state_init")


def swe_batch_run(batch, dev, params, state, n_steps: int, stats=None, stream=None) -> int:
    """Queue n_steps steps of every scenario; with a stats array (one swe_run_stats per
    scenario) synchronise and return the first failing scenario's status."""
    rc = lib.swe_batch_run(batch, C.byref(dev), C.byref(params), C.byref(state), n_steps,
                           None if stats is None else C.cast(stats, C.c_void_p), stream)
    if rc in (SWE_EINVAL, SWE_EDEVICE, SWE_EMESH, SWE_EUNSUPPORTED):
        _check(rc, "swe_batch_run")
    return rc


def swe_adjoint_workspace_bytes(mesh, n_steps: int, ckpt_every: int) -> int:
    b = C.c_int64()
    _check(lib.swe_adjoint_workspace_bytes(mesh, n_steps, ckpt_every, C.byref(b)),
           "swe_adjoint_workspace_bytes")
    return int(b.value)


def swe_adjoint(mesh, dm, params, state, n_steps, dt_seq, loss, ckpt_every, grads, ws,
                ws_bytes, stream=None) -> float:
    """Loss and gradients of a replayed run (see include/swe.h); returns the loss."""
    j = C.c_double()
    _check(lib.swe_adjoint(mesh, C.byref(dm), C.byref(params), C.byref(state), n_steps, dt_seq,
                           C.byref(loss), ckpt_every, C.byref(grads), C.byref(j), ws, ws_bytes,
                           stream), "swe_adjoint")
    return j.value


def swe_tune(mesh, dm, params, state, n_steps: int, stream=None) -> swe_tune_result:
    out = swe_tune_result()
    _check(lib.swe_tune(mesh, C.byref(dm), C.byref(params), C.byref(state), n_steps,
                        C.byref(out), stream), "swe_tune")
    return out


def swe_tune_get(device: int, dtype: int, n_cells: int) -> swe_tune_result:
    out = swe_tune_result()
    _check(lib.swe_tune_get(device, dtype, n_cells, C.byref(out)), "swe_tune_get")
    return out


def swe_tune_set(device: int, dtype: int, n_cells: int, r: swe_tune_result) -> None:
    _check(lib.swe_tune_set(device, dtype, n_cells, C.byref(r)), "swe_tune_set")


def swe_adjoint_timings() -> tuple[float, float]:
    """(forward_ms, reverse_ms) of this thread's last swe_adjoint call."""
    f, r = C.c_double(), C.c_double()
    _check(lib.swe_adjoint_timings(C.byref(f), C.byref(r)), "swe_adjoint_timings")
    return f.value, r.value


def swe_mesh_create_shard(full, c0: int, c1: int) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib.swe_mesh_create_shard(full, c0, c1, C.byref(out)), "swe_mesh_create_shard")
    return out


def swe_halo_pack(dtype, n, idx, h, hu, hv, buf, stream=None) -> None:
    _check(lib.swe_halo_pack(dtype, n, idx, h, hu, hv, buf, stream), "swe_halo_pack")


def swe_halo_unpack(dtype, n, idx, buf, h, hu, hv, stream=None) -> None:
    _check(lib.swe_halo_unpack(dtype, n, idx, buf, h, hu, hv, stream), "swe_halo_unpack")


def swe_shard_dt_combine(ctrls, stream=None) -> None:
    arr = (C.c_void_p * len(ctrls))(*ctrls)
    _check(lib.swe_shard_dt_combine(arr, len(ctrls), stream), "swe_shard_dt_combine")
