"""MI355X (gfx950) implementation of one explicit step of the cell-centred HLLC finite-volume
shallow-water solver of Zaoui (EDF R&D, 2016): HIP kernels behind the C ABI of
include/swe.h, with torch providing device memory and streams.
"""
from ._abi import (  # noqa: F401
    EXPORTS, LIB_PATH, SWE_ARR_C2N, SWE_ARR_NBR, SWE_ARR_NODE_PERM, SWE_ARR_PERM, SWE_ARR_XY,
    SWE_AUTO, SWE_CELL, SWE_CTRL_BYTES, SWE_EDEVICE, SWE_EDRY, SWE_EINVAL, SWE_EMESH, SWE_ENONFINITE,
    SWE_EUNSUPPORTED, SWE_F32, SWE_F64, SWE_MAX_INFLOW, SWE_MORTON, SWE_OK, SWE_TILE, SWE_TILED,
    SWE_WALL, SweError,
    lib, swe_dev_mesh, swe_flux_eval, swe_last_error, swe_mesh_create, swe_mesh_destroy,
    swe_mesh_export, swe_mesh_info, swe_mesh_info_get, swe_params, swe_read_stats, swe_run,
    swe_run_stats, swe_state, swe_state_init, swe_step, swe_workspace_bytes, swe_batch_create,
    swe_batch_destroy, swe_batch_export, swe_batch_info_get, swe_batch_run,
    swe_batch_state_init, swe_batch_workspace_bytes, swe_adjoint, swe_adjoint_timings, swe_adjoint_workspace_bytes,
    swe_grads, swe_loss, swe_tune, swe_tune_get, swe_tune_result, swe_tune_set,
    swe_mesh_create_shard, swe_halo_pack, swe_halo_unpack, swe_shard_dt_combine, SWE_SHARD,
    SWE_ARR_GLOBAL, SWE_INDEX64, SWE_EXACT, SWE_HILBERT, SWE_TILE_64, SWE_TILE_128, SWE_TILE_512,
    swe_run_static)
from .solver import Batch, BatchSolver, Mesh, Solver  # noqa: F401
from .adjoint import AdjointLoss, Calibration  # noqa: F401
from . import tune  # noqa: F401
from .shard import ShardedSolver  # noqa: F401


def require_gpu() -> None:
    """Raise unless a GPU is visible (the library has no CPU implementation)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libswe needs an AMD GPU (gfx950); none is visible")
