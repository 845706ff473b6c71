"""Every configuration at its configured size against the oracle, every cell.

Section 3 of the paper checks the GPU results against the CPU code at t = T_s on grids of
Table 2's scale.  Here the FP64 oracle runs on this host inside the test (once per module and
configuration) and the HIP path runs in the launch configuration the benchmark times:

- configurations 2 (1,000,000 triangles, 1,000 steps) and 3 (10,000,000 triangles, 500 steps):
  FP64 (both arithmetic modes) every field within 1e-12 of its scale, identical wet/dry masks,
  clamp and step counts;
  FP32 against the oracle started from the same float-rounded inputs (bed, roughness and state
  rounded to float32 and back), h within 1e-5 of max h, momentum within the bound of
  tests/parity.py (fp32_momentum_bound), masks identical outside the band of 1e-5 max h
  around the dry threshold;
- configuration 4 (the 256-scenario ensemble, 2,000 steps, one batched launch per step): 32
  scenarios stratified by size compared on every cell, FP64 as above, FP32 as above but with
  the depth tolerance of a moving front over 2,000 steps (fp32_front_tol);
- configuration 5 (250,000-cell calibration, 2,000 steps, checkpoints every 50): the loss
  against the oracle's, the gradient's dot products with random directions in n and z
  against the oracle's tangent-linear derivative, and central differences of the GPU loss on
  cells whose perturbed runs keep the base run's branches (the oracle's branch signature).
"""
import math
import os

import numpy as np
import pytest

import gen
import oracle
from parity import (TOL_F32, TOL_F64, errors, float_rounded, fp32_errors, mask_mismatch,
                    run_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def store():
    return {}


def _case(store, k):
    key = ("case", k)
    if key not in store:
        store[key] = gen.config(k)
    return store[key]


def _oracle(store, k, rounded):
    """The oracle's final state of configuration k (from float-rounded inputs if `rounded`)."""
    key = ("oracle", k, rounded)
    if key not in store:
        case = _case(store, k)
        c = float_rounded(case) if rounded else case
        mk = ("omesh", k)
        if mk not in store:
            store[mk] = oracle.Mesh(case.xy, case.tri, case.edge_tag)
        rc, h, hu, hv, dts, st = oracle.run_case(c, mesh=store[mk])
        assert rc == 0
        store[key] = (h, hu, hv, st)
    return store[key]


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("k", [2, 3])
def test_fp64_every_cell_at_the_configured_size(gpu, store, k, exact):
    """Both FP64 arithmetic modes: the fast forms and SWE_EXACT (correctly rounded division and
    square root)."""
    case = _case(store, k)
    h_o, hu_o, hv_o, st_o = _oracle(store, k, False)
    rc, st, h, hu, hv = run_gpu(case, "f64", exact=exact)
    e = errors(case, (h, hu, hv), (h_o, hu_o, hv_o))
    mism, _ = mask_mismatch(case, h, h_o)
    mode = "f64 exact" if exact else "f64"
    print(f"config {k} {mode}, {case.n_cells} cells x {case.steps} steps: errors h {e[0]:.2e} "
          f"hu {e[1]:.2e} hv {e[2]:.2e}; wet/dry mismatches {mism}; t {st['t']!r} vs "
          f"{st_o['t']!r}; clamps {st['clamps']} vs {st_o['clamps']}", flush=True)
    assert rc == 0 and st["steps"] == st_o["steps"] == case.steps
    assert max(e) <= TOL_F64
    assert mism == 0
    assert st["clamps"] == st_o["clamps"]
    assert st["t"] == pytest.approx(st_o["t"], rel=TOL_F64)


@pytest.mark.parametrize("k", [2, 3])
def test_fp32_every_cell_against_the_oracle_of_the_float_inputs(gpu, store, k):
    case = _case(store, k)
    h_o, hu_o, hv_o, st_o = _oracle(store, k, True)
    rc, st, h, hu, hv = run_gpu(case, "f32")
    e_h, e_q = fp32_errors(case, (h, hu, hv), (h_o, hu_o, hv_o))
    band = TOL_F32 * float(np.abs(h_o).max())
    mism, exempt = mask_mismatch(case, h, h_o, band)
    total, _ = mask_mismatch(case, h, h_o)
    print(f"config {k} f32, {case.n_cells} cells x {case.steps} steps: h error {e_h:.2e} of "
          f"max h, momentum error {e_q:.3f} of its bound; wet/dry mismatches {mism} outside "
          f"the band ({exempt} cells in it, {total} mismatches in all); t {st['t']!r} vs "
          f"{st_o['t']!r}", flush=True)
    assert rc == 0 and st["steps"] == st_o["steps"] == case.steps
    assert e_h <= TOL_F32 and e_q <= 1.0
    assert mism == 0
    assert st["t"] == pytest.approx(st_o["t"], rel=TOL_F32)


# ------------------------------------------------------------------ configuration 4

N_ENSEMBLE_CHECKED = 32


def fp32_front_tol(steps, courant):
    """Depth tolerance (relative to max h) of an FP32 run of `steps` steps with moving fronts:
    the bores the inflows drive move at a speed FP32 forms with a relative error of its unit
    roundoff u = 2^-24, so each step a front lands up to C u of a cell away from the oracle's
    (C the Courant number) and after N steps up to N C u of a cell; across a front the depth
    changes by up to max h per cell, so the depth there differs by up to N C u max h.  The
    stated 1e-5 of max h holds where that is smaller."""
    return max(TOL_F32, steps * courant * 2.0 ** -24)


@pytest.fixture(scope="module")
def ensemble(gpu):
    cases = gen.ensemble(256)
    order = np.argsort([c.n_cells for c in cases], kind="stable")
    # every eighth scenario by size: the smallest, the largest and everything between
    picked = [int(order[i]) for i in
              np.linspace(0, len(cases) - 1, N_ENSEMBLE_CHECKED).round().astype(np.int64)]
    meshes = [gpu.Mesh(c.xy, c.tri, c.edge_tag) for c in cases]
    batch = gpu.Batch(meshes)
    return cases, picked, batch


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ensemble_at_2000_steps_against_the_oracle(gpu, ensemble, dtype):
    cases, picked, batch = ensemble
    steps = cases[0].steps
    bs = gpu.BatchSolver(batch, cases, dtype=dtype)
    rc, st = bs.run(steps)
    assert rc == 0
    worst = [0.0, 0.0, 0.0]
    total_mism = 0
    for s in picked:
        case = cases[s]
        c = float_rounded(case) if dtype == "f32" else case
        rc_o, h_o, hu_o, hv_o, _, st_o = oracle.run_case(c)
        assert rc_o == 0 and st[s]["steps"] == st_o["steps"] == steps
        h, hu, hv = bs.numpy_state(s)
        if dtype == "f64":
            e = errors(case, (h, hu, hv), (h_o, hu_o, hv_o))
            mism, _ = mask_mismatch(case, h, h_o)
            tol = TOL_F64
            assert st[s]["clamps"] == st_o["clamps"]
        else:
            e_h, e_q = fp32_errors(case, (h, hu, hv), (h_o, hu_o, hv_o))
            e = (e_h, e_q, 0.0)
            mism, _ = mask_mismatch(case, h, h_o, TOL_F32 * float(np.abs(h_o).max()))
            tol = fp32_front_tol(steps, case.courant)
            assert e_q <= 1.0, (s, case.n_cells, e_h, e_q)
        worst = [max(a, b) for a, b in zip(worst, e)]
        total_mism += mism
        assert e[0] <= tol and (dtype == "f32" or max(e) <= tol), (s, case.n_cells, e)
        assert mism == 0, (s, mism)
        assert st[s]["t"] == pytest.approx(st_o["t"], rel=tol)
    what = ("h, hu, hv relative" if dtype == "f64" else
            f"h relative to max h (tolerance {fp32_front_tol(steps, cases[0].courant):.2e}), "
            "momentum as a fraction of its bound, -")
    print(f"ensemble {dtype}: {len(picked)} of {len(cases)} scenarios "
          f"({min(cases[s].n_cells for s in picked)} to {max(cases[s].n_cells for s in picked)} "
          f"cells) x {steps} steps: worst errors ({what}) {worst[0]:.2e} {worst[1]:.2e} "
          f"{worst[2]:.2e}; wet/dry mismatches {total_mism}", flush=True)


# ------------------------------------------------------------------ configuration 5

@pytest.fixture(scope="module")
def calibration(gpu):
    case = gen.config(5)
    om = oracle.Mesh(case.xy, case.tri)
    dts, obs = oracle.observations(case, om)
    mesh = gpu.Mesh(case.xy, case.tri)
    ex = case.extra
    calib = gpu.Calibration(mesh, dts, ex["gauges"], obs, every=ex["obs_every"],
                            ckpt_every=ex["ckpt_every"])
    j, grads = calib.run(case.n, case.z, case.h, case.hu, case.hv)
    return case, om, dts, obs, calib, j, grads


def test_calibration_loss_at_the_configured_size(calibration):
    """J = sum of squared gauge misfits r; with every gauge depth within delta = 1e-12 of the
    depth scale of the oracle's, |J - J_o| <= 2 delta sum|r| + M delta^2
    <= 2 delta sqrt(M J_o) + M delta^2 over the M observations (Cauchy-Schwarz)."""
    case, om, dts, obs, calib, j, grads = calibration
    ex = case.extra
    jo = oracle.run_loss(om, case.z, case.n, case.h, case.hu, case.hv, dts, ex["gauges"],
                         ex["obs_every"], obs)
    m = obs.size
    delta = TOL_F64 * max(float(np.abs(case.h).max()), float(np.abs(obs).max()))
    bound = 2 * delta * math.sqrt(m * jo) + m * delta * delta
    print(f"calibration: {case.n_cells} cells x {case.steps} steps, J {j!r} vs oracle {jo!r} "
          f"(difference {abs(j - jo):.2e}, bound {bound:.2e})", flush=True)
    assert jo > 0 and abs(j - jo) <= bound


@pytest.mark.parametrize("which", ["n", "z"])
def test_calibration_gradient_dot_products_at_the_configured_size(calibration, which):
    case, om, dts, obs, calib, j, grads = calibration
    ex = case.extra
    k = ["n", "z", "h", "hu", "hv"].index(which)
    v = np.random.default_rng(500 + k).normal(size=case.n_cells)
    jo, djo = oracle.run_tl(om, case.z, case.n, case.h, case.hu, case.hv, dts, ex["gauges"],
                            ex["obs_every"], obs, **{"d" + which: v})
    adj = float(np.dot(grads[k], v))
    print(f"calibration d{which}: <grad, v> = {adj!r}, oracle tangent dJ[v] = {djo!r} "
          f"(relative difference {abs(adj - djo) / abs(djo):.2e})", flush=True)
    assert adj == pytest.approx(djo, rel=1e-9)


def test_calibration_central_differences_away_from_switches(calibration):
    """Central differences (eps = 1e-6) of the GPU loss in n on 32 random wet cells against
    the adjoint's dJ/dn, compared where both perturbed runs keep the base run's branches: the
    oracle's branch signature of the run with n + eps e_c and with n - eps e_c equals the base
    run's (a signature covers every branch of every edge and cell at every step)."""
    case, om, dts, obs, calib, j, grads = calibration
    ex = case.extra
    args = (dts, ex["gauges"], ex["obs_every"], obs)
    _, s0 = oracle.run_loss_sig(om, case.z, case.n, case.h, case.hu, case.hv, *args)
    rng = np.random.default_rng(7)
    cells = rng.choice(np.flatnonzero(case.h > 1e-2), size=32, replace=False)
    dn = grads[0]
    eps = 1e-6

    def perturbed(c):
        n_p, n_m = case.n.copy(), case.n.copy()
        n_p[c] += eps
        n_m[c] -= eps
        return n_p, n_m

    def keeps_branches(c):
        k = all(oracle.run_loss_sig(om, case.z, nn, case.h, case.hu, case.hv, *args)[1] == s0
                for nn in perturbed(c))
        print(f"cell {c}: {'keeps' if k else 'changes'} the base run's branches", flush=True)
        return k

    # the oracle's runs are independent C calls (ctypes releases the GIL)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        keep = list(pool.map(keeps_branches, cells))
    kept, bad = 0, []
    for c, k in zip(cells, keep):
        if not k:
            continue
        n_p, n_m = perturbed(c)
        kept += 1
        jp, _ = calib.run_device(*[_dev(calib, a) for a in (n_p, case.z, case.h, case.hu, case.hv)])
        jm, _ = calib.run_device(*[_dev(calib, a) for a in (n_m, case.z, case.h, case.hu, case.hv)])
        fd = (jp - jm) / (2 * eps)
        if abs(fd - dn[c]) > 1e-6 * np.abs(dn).max() + 1e-4 * abs(dn[c]):
            bad.append((int(c), fd, float(dn[c])))
    print(f"calibration FD: {kept} of {len(cells)} cells keep the base run's branches; "
          f"max |dJ/dn| {np.abs(dn).max():.3e}; disagreements {bad}", flush=True)
    assert kept >= 16 and not bad


def _dev(calib, a):
    import torch
    return torch.as_tensor(np.asarray(a, np.float64), device=calib.mesh.device)
