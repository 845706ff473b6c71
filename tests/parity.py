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


def float_rounded(case):
    """The case with bed, roughness, initial state and inflow discharges rounded to float32
    (and held in float64): the inputs an FP32 run actually starts from.  The mesh is kept."""
    import copy
    c = copy.copy(case)
    r = lambda a: None if a is None else np.asarray(a, np.float32).astype(np.float64)
    c.z, c.n, c.h, c.hu, c.hv = r(case.z), r(case.n), r(case.h), r(case.hu), r(case.hv)
    c.inflow_q = r(case.inflow_q)
    return c


def fp32_momentum_bound(case, ora_fields):
    """Absolute bound on the momentum error of an FP32 run against the FP64 oracle started
    from the same float-rounded inputs (`float_rounded`).

    The FP32 target holds depth errors to delta = 1e-5 max h.  A depth (free-surface) error
    moves as gravity waves, whose momentum perturbation is c times their surface perturbation
    (c = sqrt(g h), from the Riemann invariants q +- c eta of the linearised equations); a
    left- and a right-going part, each within delta, give momentum errors up to
    2 c_max delta, c_max = sqrt(g max h).  Rounding of the momentum's own arithmetic adds
    1e-5 of its magnitude (the same relative target as the depth)."""
    h_o, hu_o, hv_o = ora_fields
    hmax = float(np.abs(h_o).max())
    delta = TOL_F32 * hmax
    qmax = float(np.sqrt(hu_o * hu_o + hv_o * hv_o).max())
    return 2.0 * math.sqrt(case.g * hmax) * delta + TOL_F32 * qmax


def fp32_errors(case, gpu_fields, ora_fields):
    """FP32 errors against the oracle of the float-rounded inputs: the depth error relative to
    max h (target 1e-5) and the largest momentum error, as a vector (hu, hv), over its bound
    `fp32_momentum_bound` (target 1)."""
    h_g, hu_g, hv_g = gpu_fields
    h_o, hu_o, hv_o = ora_fields
    e_h = float(np.abs(h_g - h_o).max()) / float(np.abs(h_o).max())
    e_q = float(np.sqrt((hu_g - hu_o) ** 2 + (hv_g - hv_o) ** 2).max())
    return e_h, e_q / fp32_momentum_bound(case, ora_fields)


def mask_mismatch(case, h_g, h_o, band=0.0):
    """Cells wet on one side and dry on the other, outside |h_o - h_dry| <= band."""
    wet_g = h_g > case.h_dry
    wet_o = h_o > case.h_dry
    exempt = np.abs(h_o - case.h_dry) <= band
    return int(((wet_g != wet_o) & ~exempt).sum()), int(exempt.sum())
