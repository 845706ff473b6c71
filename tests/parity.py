"""Shared helpers of the GPU parity tests: run a case on the HIP path and on the oracle, and
compare them with the error norm of the tolerance reading (per field: max abs difference over
max(|oracle|, floor); floor 0 for h, 1e-3 max h sqrt(g max h) for momentum)."""
from __future__ import annotations

import math

import numpy as np

import oracle

TOL_F64 = 1e-12
TOL_F32 = 1e-5


def run_gpu(case, dtype="f64", steps=None, morton=True, t_end=0.0, dt_seq=None, mesh=None,
            variant="auto", exact=False):
    import torch

    import paper_1807_00672_amd as swe
    m = mesh or swe.Mesh(case.xy, case.tri, case.edge_tag, morton=morton)
    s = swe.Solver(m, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype, g=case.g,
                   courant=case.courant, h_dry=case.h_dry, inflow_q=case.inflow_q, t_end=t_end,
                   variant=variant, exact=exact)
    seq = None if dt_seq is None else torch.as_tensor(dt_seq, dtype=torch.float64,
                                                      device=m.device)
    rc, st = s.run(case.steps if steps is None else steps, dt_seq=seq)
    h, hu, hv = s.numpy_state()
    return rc, st, h, hu, hv


def quarter_turn(case):
    """The case turned a quarter about the origin: (x, y) -> (-y, x), exact in floating point,
    with the initial momentum turned alike."""
    import copy
    c = copy.copy(case)
    c.xy = np.ascontiguousarray(np.stack([-case.xy[:, 1], case.xy[:, 0]], axis=1))
    c.hu, c.hv = -case.hv, case.hu.copy()
    return c


def run_oracle(case, steps=None, t_end=0.0, dt_seq=None, mesh=None):
    return oracle.run_case(case, steps=steps, t_end=t_end, dt_seq=dt_seq, mesh=mesh)


def errors(case, gpu_fields, ora_fields):
    h_o, hu_o, hv_o = ora_fields
    h_g, hu_g, hv_g = gpu_fields
    hmax = float(np.abs(h_o).max())
    floor = 1e-3 * hmax * math.sqrt(case.g * hmax)
    e_h = float(np.abs(h_g - h_o).max()) / hmax
    e_hu = float(np.abs(hu_g - hu_o).max()) / max(float(np.abs(hu_o).max()), floor)
    e_hv = float(np.abs(hv_g - hv_o).max()) / max(float(np.abs(hv_o).max()), floor)
    return e_h, e_hu, e_hv


def fp32_momentum_tol(case, h_o):
    """Absolute momentum tolerance of the FP32 path.

    Storing the bed and the depth in float moves the free surface eta = h + z by up to
    eps32 * max|eta|, which the hydrostatic reconstruction sees as a surface slope: the
    discrete lake at rest is lost and velocities of order sqrt(g * eps32 * max|eta|) appear
    (gravity-wave speed of that surface error).  Momentum errors of that velocity times the
    largest depth are inherent to the FP32 state, not to the kernels."""
    eps32 = float(np.finfo(np.float32).eps)
    hmax = float(np.abs(h_o).max())
    eta_max = float(np.abs(case.z).max()) + hmax
    return hmax * math.sqrt(case.g * eps32 * eta_max)


def mask_mismatch(case, h_g, h_o, band=0.0):
    """Cells wet on one side and dry on the other, outside |h_o - h_dry| <= band."""
    wet_g = h_g > case.h_dry
    wet_o = h_o > case.h_dry
    exempt = np.abs(h_o - case.h_dry) <= band
    return int(((wet_g != wet_o) & ~exempt).sum()), int(exempt.sum())
