"""Launch autotuning (swe_tune): which step kernel variant and workgroup order run fastest for
a mesh size class on this device, remembered for SWE_AUTO; which tile size (the step kernels'
workgroup size, a property of the mesh: one mesh per size) is fastest, remembered for
Mesh(tile="auto"); optional persistence as JSON keyed by device name, precision and size class,
and a choice among Morton, Hilbert and input cell order."""
from __future__ import annotations

import json
import os

import torch

from . import _abi as A
from .solver import Mesh, Solver

_DT = {"f64": A.SWE_F64, "f32": A.SWE_F32}
_VAR = {"auto": A.SWE_AUTO, "cell": A.SWE_CELL, "tiled": A.SWE_TILED}
_recorded: dict[tuple[str, int], dict] = {}   # (dtype, size class) -> result, this process


def size_class(n_cells: int) -> int:
    return int(n_cells).bit_length() - 1


def _device_index(mesh: Mesh) -> int:
    return mesh.device.index if mesh.device.index is not None else torch.cuda.current_device()


def tune(mesh: Mesh, z, n, h, hu, hv, dtype: str = "f64", steps: int = 20, **solver_kw) -> dict:
    """Time every variant x workgroup order on a scratch state of this setup (the caller's
    arrays are not touched) and record the fastest for SWE_AUTO.  Returns the timings."""
    s = Solver(mesh, z, n, h, hu, hv, dtype=dtype, **solver_kw)
    with torch.cuda.device(mesh.device):
        r = A.swe_tune(mesh.handle, mesh.dev, s.params, s.state, steps, None).as_dict()
    _recorded[(dtype, size_class(mesh.n_cells))] = r
    return r


def tuning(dtype: str, n_cells: int, device: int | None = None) -> dict | None:
    """The recorded choice for this device, precision and size class, or None."""
    dev = torch.cuda.current_device() if device is None else device
    r = A.swe_tune_get(dev, _DT[dtype], n_cells).as_dict()
    return None if r["variant"] == "auto" else r


def forget(dtype: str, n_cells: int, device: int | None = None) -> None:
    dev = torch.cuda.current_device() if device is None else device
    A.swe_tune_set(dev, _DT[dtype], n_cells, A.swe_tune_result())


def save(path: str) -> None:
    """Add this process's tuning results to a JSON file under this device's name."""
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    entries = data.setdefault(name, {})
    for (dt, cls), r in _recorded.items():
        entries[f"{dt}:{cls}"] = {"variant": r["variant"], "xcd_remap": r["xcd_remap"],
                                  "tile": r.get("tile", A.SWE_TILE),
                                  "ms_per_step": r["ms_per_step"]}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(path: str) -> int:
    """Record the choices a JSON file holds for this device's name; returns how many."""
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    with open(path) as f:
        entries = json.load(f).get(name, {})
    dev = torch.cuda.current_device()
    for key, e in entries.items():
        dt, cls = key.split(":")
        r = A.swe_tune_result()
        r.variant = _VAR[e["variant"]]
        r.xcd_remap = 1 if e["xcd_remap"] else 0
        r.tile_cells = int(e.get("tile", A.SWE_TILE))
        A.swe_tune_set(dev, _DT[dt], 1 << int(cls), r)
    return len(entries)


def tune_order(xy, tri, z, n, h, hu, hv, edge_tag=None, dtype: str = "f64",
               steps: int = 20, orders=("morton", "hilbert", "input"),
               **solver_kw) -> tuple[str, dict]:
    """Build the mesh in each cell order, tune each, and return (the fastest order, the
    timings of every order).  The fastest order's best variant stays recorded."""
    res = {}
    for order in orders:
        m = Mesh(xy, tri, edge_tag, order=order)
        res[order] = tune(m, z, n, h, hu, hv, dtype, steps, **solver_kw)
    order = min(res, key=lambda k: _best_ms(res[k]))
    _record(res[order], dtype, len(tri))   # the order tuned last may not be the fastest
    return order, res


def _best_ms(r: dict) -> float:
    return min(v for v in r["ms_per_step"].values() if v > 0)


def _record(r: dict, dtype: str, n_cells: int) -> None:
    rr = A.swe_tune_result()
    rr.variant = _VAR[r["variant"]]
    rr.xcd_remap = 1 if r["xcd_remap"] else 0
    rr.tile_cells = int(r.get("tile", A.SWE_TILE))
    A.swe_tune_set(torch.cuda.current_device(), _DT[dtype], n_cells, rr)
    _recorded[(dtype, size_class(n_cells))] = r


def tune_tiles(xy, tri, z, n, h, hu, hv, edge_tag=None, dtype: str = "f64", steps: int = 20,
               tiles=(64, 128, 256, 512), order: str = "morton", **solver_kw) -> tuple[int, dict]:
    """Build the mesh with each tile size (cells per workgroup of the step kernels), tune each
    (variant x workgroup order, swe_tune), and record the fastest tile size with its variant
    and order for this device, precision and size class: Mesh(..., tile="auto") then builds
    with it and SWE_AUTO launches its variant.  Returns (the fastest tile size, the timings of
    every size)."""
    res = {}
    for tile in tiles:
        m = Mesh(xy, tri, edge_tag, order=order, tile=tile)
        res[tile] = tune(m, z, n, h, hu, hv, dtype, steps, **solver_kw)
        del m
        torch.cuda.empty_cache()
    best = min(res, key=lambda t: _best_ms(res[t]))
    _record(res[best], dtype, len(tri))
    return best, res
