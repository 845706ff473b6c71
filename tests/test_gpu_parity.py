"""HIP path against the FP64 oracle, element by element, on seeded inputs.

The oracle follows section 2 of the paper (eq. 4 over the three edges of each triangle, HLLC
with hydrostatic reconstruction, semi-implicit friction, CFL with Courant 0.7).  Tolerances:
FP64 1e-12 relative per field; FP32 1e-5 relative to max h, wet/dry masks identical outside a
band of 1e-5 max h around the dry threshold; step counts identical.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from parity import (TOL_F32, TOL_F64, errors, float_rounded, fp32_errors, mask_mismatch, quarter_turn,
                    run_gpu, run_oracle)

pytestmark = pytest.mark.gpu


def _rand_edges(rng, n, dry_frac=0.2):
    h = rng.uniform(0.0, 3.0, n)
    h[rng.random(n) < dry_frac] = 0.0
    h[rng.random(n) < 0.05] = 0.5e-6
    return h, rng.uniform(-6, 6, n) * h, rng.uniform(-6, 6, n) * h


@pytest.mark.parametrize("exact", [True, False])
@pytest.mark.parametrize("wall", [False, True])
def test_flux_matches_oracle_bitwise_in_fp64(gpu, wall, exact):
    """SWE_EXACT: the same bits as the oracle.  Default (fast forms): the HLL quotients and the
    unit normal are refined to within an ulp, but each velocity is a momentum times the depth's
    reciprocal, within 1.5 ulp, so the normal velocity q = u n_x + v n_y may be off by
    2 eps |U| (|U| the larger velocity component of the edge's two sides, cancellation in the
    sum included); the flux depends on q with |dF/dq| <= 4 (|U| + c) h (the terms h q^2 and
    S h q of the HLL average, c = sqrt(g h), h the larger depth).  Per edge, the error is then
    within 64 eps of the flux scale 1 + |F| (the HLLC arithmetic's own rounding) plus
    8 eps |U| (|U| + c) h."""
    import torch
    rng = np.random.default_rng(11)
    n = 1 << 20
    hl, hul, hvl = _rand_edges(rng, n)
    hr, hur, hvr = _rand_edges(rng, n)
    zl = rng.uniform(-1, 1, n)
    zr = np.where(rng.random(n) < 0.3, zl, rng.uniform(-1, 1, n))
    th = rng.uniform(0, 2 * math.pi, n)
    nx, ny = np.cos(th), np.sin(th)
    if wall:
        f_o, p_o = oracle.wall(hl, hul, hvl, nx, ny)
    else:
        f_o, p_o, _ = oracle.interface(hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny)
    d = {k: torch.from_numpy(v).cuda() for k, v in dict(hl=hl, hul=hul, hvl=hvl, zl=zl, hr=hr,
                                                        hur=hur, hvr=hvr, zr=zr, nx=nx,
                                                        ny=ny).items()}
    f = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    p = torch.empty(n, dtype=torch.float64, device="cuda")
    P = lambda t: t.data_ptr()
    gpu.swe_flux_eval(gpu.SWE_F64, n, 9.81, 1e-6, P(d["hl"]), P(d["hul"]), P(d["hvl"]),
                      P(d["zl"]), None if wall else P(d["hr"]), None if wall else P(d["hur"]),
                      None if wall else P(d["hvr"]), None if wall else P(d["zr"]), P(d["nx"]),
                      P(d["ny"]), P(f), P(p), flags=gpu.SWE_EXACT if exact else 0)
    torch.cuda.synchronize()
    f_g = f.cpu().numpy().reshape(n, 3)
    if exact:
        assert np.array_equal(f_g, f_o)
        assert np.array_equal(p.cpu().numpy(), p_o)
        return
    eps = np.finfo(np.float64).eps
    scale = 1.0 + np.abs(f_o).max(axis=1)
    dif = np.abs(f_g - f_o).max(axis=1)
    vel = lambda h, q: np.where(h > 1e-6, q / np.where(h > 1e-6, h, 1.0), 0.0)
    if wall:
        umax = np.maximum(np.abs(vel(hl, hul)), np.abs(vel(hl, hvl)))
        hmax = hl
    else:
        umax = np.max(np.abs([vel(hl, hul), vel(hl, hvl), vel(hr, hur), vel(hr, hvr)]), axis=0)
        hmax = np.maximum(hl, hr)
    bound = 64 * eps * scale + 8 * eps * umax * (umax + np.sqrt(9.81 * hmax)) * hmax
    print(f"fast FP64 flux: max error {(dif / scale).max():.3e} of the flux scale; "
          f"largest fraction of the per-edge bound {(dif / bound).max():.3f}")
    assert (dif <= bound).all()
    assert np.array_equal(p.cpu().numpy(), p_o)   # the bed correction has no division


def test_flux_fp32_is_close(gpu):
    import torch
    rng = np.random.default_rng(12)
    n = 1 << 18
    hl, hul, hvl = _rand_edges(rng, n)
    hr, hur, hvr = _rand_edges(rng, n)
    zl = rng.uniform(-1, 1, n)
    zr = rng.uniform(-1, 1, n)
    th = rng.uniform(0, 2 * math.pi, n)
    nx, ny = np.cos(th), np.sin(th)
    f_o, p_o, _ = oracle.interface(hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny)
    args = [torch.from_numpy(v.astype(np.float32)).cuda()
            for v in (hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny)]
    f = torch.empty(3 * n, dtype=torch.float32, device="cuda")
    p = torch.empty(n, dtype=torch.float32, device="cuda")
    gpu.swe_flux_eval(gpu.SWE_F32, n, 9.81, 1e-6, *[a.data_ptr() for a in args], f.data_ptr(),
                      p.data_ptr())   # FP32 has one arithmetic; SWE_EXACT concerns FP64
    torch.cuda.synchronize()
    f_g = f.cpu().numpy().reshape(n, 3).astype(np.float64)
    # inputs were rounded to float: compare against the oracle on the rounded inputs
    r = [a.cpu().numpy().astype(np.float64) for a in args]
    f_r, p_r, _ = oracle.interface(*r)
    scale = 1.0 + np.abs(f_r).max(axis=1)
    # cells at the dry threshold may legitimately switch branch in float
    ok = (np.abs(r[0] - 1e-6) > 1e-8) & (np.abs(r[4] - 1e-6) > 1e-8)
    assert (np.abs(f_g - f_r).max(axis=1)[ok] / scale[ok]).max() < 5e-5


@pytest.mark.parametrize("variant", ["tiled", "cell"])
def test_exact_fp64_reproduces_the_oracle_bitwise_without_friction(gpu, variant):
    """With SWE_EXACT every operation of the step is the oracle's, in the oracle's order; with
    n = 0 (config 1) no cube root is taken, so the whole run is bit for bit the oracle's."""
    import paper_1807_00672_amd as swe
    case = gen.small(1)
    rc_o, h_o, hu_o, hv_o, dts, st_o = run_oracle(case)
    m = swe.Mesh(case.xy, case.tri)
    s = swe.Solver(m, case.z, case.n, case.h, case.hu, case.hv, dtype="f64", variant=variant,
                   exact=True)
    rc, st = s.run(case.steps)
    assert rc == rc_o == 0 and st["t"] == st_o["t"]
    for a, b in zip(s.numpy_state(), (h_o, hu_o, hv_o)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["tiled", "cell"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_fp64_parity_small_configs(gpu, k, variant):
    case = gen.small(k)
    rc_o, *ora, dts, st_o = run_oracle(case)
    rc_g, st_g, *g = run_gpu(case, "f64", variant=variant)
    assert rc_o == 0 and rc_g == 0
    assert st_g["steps"] == st_o["steps"] == case.steps
    e = errors(case, g, ora)
    print(f"config {k} small fp64 {variant}: errors {e}, exact h {np.mean(g[0] == ora[0]):.4f}, "
          f"t gpu {st_g['t']!r} oracle {st_o['t']!r}")
    assert max(e) <= TOL_F64
    assert st_g["t"] == pytest.approx(st_o["t"], rel=TOL_F64)
    assert mask_mismatch(case, g[0], ora[0])[0] == 0
    assert st_g["clamps"] == st_o["clamps"]


@pytest.mark.parametrize("variant", ["tiled", "cell"])
@pytest.mark.parametrize("k", [2, 3])
def test_fp32_parity_small_configs(gpu, k, variant):
    """FP32 against the oracle started from the same float-rounded inputs: h within 1e-5 of
    max h, momentum within its bound (tests/parity.py: fp32_momentum_bound)."""
    case = gen.small(k)
    rc_o, *ora, dts, st_o = run_oracle(float_rounded(case))
    rc_g, st_g, *g = run_gpu(case, "f32", variant=variant)
    assert rc_o == 0 and rc_g == 0 and st_g["steps"] == st_o["steps"]
    hmax = np.abs(ora[0]).max()
    e_h, e_q = fp32_errors(case, g, ora)
    mism, exempt = mask_mismatch(case, g[0], ora[0], band=TOL_F32 * hmax)
    print(f"config {k} small fp32 {variant}: h error {e_h:.2e} of max h, momentum error "
          f"{e_q:.3f} of its bound; mask mismatches {mism}, exempt {exempt}")
    assert e_h <= TOL_F32
    assert e_q <= 1.0
    assert mism == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tiled_and_per_cell_kernels_agree_bitwise(gpu, dtype):
    """Both step kernels evaluate every contribution with the same operations in the same
    order; only where each interface is computed differs."""
    case = gen.small(3)
    a = run_gpu(case, dtype, steps=80, variant="tiled")
    b = run_gpu(case, dtype, steps=80, variant="cell")
    for x, y in zip(a[2:], b[2:]):
        assert np.array_equal(x, y)
    import paper_1807_00672_amd as swe
    m = swe.Mesh(case.xy, case.tri)
    s = swe.Solver(m, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype, xcd_remap=False)
    s.run(80)
    for x, y in zip(s.numpy_state(), a[2:]):
        assert np.array_equal(x, y)
    # the tiled kernel's 64-bit index arithmetic (meshes beyond 4 GiB arrays) on a small mesh
    s = swe.Solver(m, case.z, case.n, case.h, case.hu, case.hv, dtype=dtype, variant="tiled",
                   index64=True)
    s.run(80)
    for x, y in zip(s.numpy_state(), a[2:]):
        assert np.array_equal(x, y)
    c = gen.ensemble_scenario(5)
    a = run_gpu(c, dtype, steps=50, variant="tiled")
    b = run_gpu(c, dtype, steps=50, variant="cell")
    for x, y in zip(a[2:], b[2:]):
        assert np.array_equal(x, y)


def test_cell_order_does_not_change_results(gpu):
    import paper_1807_00672_amd as swe
    case = gen.small(2)
    a = run_gpu(case, "f64", steps=100, morton=True)
    b = run_gpu(case, "f64", steps=100, morton=False)
    c = run_gpu(case, "f64", steps=100, mesh=swe.Mesh(case.xy, case.tri, order="hilbert"))
    for x, y, w in zip(a[2:], b[2:], c[2:]):
        assert np.array_equal(x, y) and np.array_equal(x, w)


def _large():
    """40,000 cells in 157 tiles: the step merges its dt partials into atomic slots that a
    fold kernel reads and resets (up to 128 tiles the step folds them itself)."""
    return gen.dam_break(nx=200, ny=100, lx=40.0, ly=20.0)


@pytest.mark.parametrize("large", [False, True])
def test_runs_are_bitwise_repeatable_and_stepwise_equal(gpu, large):
    import paper_1807_00672_amd as swe
    case = _large() if large else gen.small(3)
    a = run_gpu(case, "f64", steps=60)
    b = run_gpu(case, "f64", steps=60)
    for x, y in zip(a[2:], b[2:]):
        assert np.array_equal(x, y)
    m = swe.Mesh(case.xy, case.tri)
    s = swe.Solver(m, case.z, case.n, case.h, case.hu, case.hv)
    for _ in range(60):
        s.step()
    for x, y in zip(s.numpy_state(), a[2:]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("large", [False, True])
def test_t_end_gives_the_oracle_step_count(gpu, large):
    case = _large() if large else gen.config(1)
    rc_o, *ora, dts, st_o = run_oracle(case, steps=100000, t_end=0.5)
    rc_g, st_g, *g = run_gpu(case, "f64", steps=1000, t_end=0.5)
    assert rc_o == 0 and rc_g == 0
    assert st_g["steps"] == st_o["steps"] and st_g["t"] == 0.5 and st_g["done"] == 1
    assert max(errors(case, g, ora)) <= TOL_F64


@pytest.mark.parametrize("large", [False, True])
def test_replayed_dt_sequence(gpu, large):
    case = _large() if large else gen.small(2)
    seq = np.full(80, 0.005 if large else 0.05)
    seq[::7] = 0.008 if large else 0.08
    rc_o, *ora, dts, st_o = run_oracle(case, steps=80, dt_seq=seq)
    rc_g, st_g, *g = run_gpu(case, "f64", steps=80, dt_seq=seq)
    assert rc_o == 0 and rc_g == 0 and st_g["steps"] == 80
    assert st_g["dt_sum"] == pytest.approx(seq.sum(), rel=1e-15)
    assert max(errors(case, g, ora)) <= TOL_F64


@pytest.mark.parametrize("variant", ["tiled", "cell"])
def test_inflow_scenario_matches_oracle(gpu, variant):
    case = gen.ensemble_scenario(3)
    rc_o, *ora, dts, st_o = run_oracle(case, steps=300)
    rc_g, st_g, *g = run_gpu(case, "f64", steps=300, variant=variant)
    assert rc_o == 0 and rc_g == 0
    assert max(errors(case, g, ora)) <= TOL_F64


def test_lake_at_rest_and_mass_on_gpu(gpu):
    case = gen.lake_at_rest()
    rc, st, h, hu, hv = run_gpu(case, "f64")
    assert rc == 0 and st["steps"] == case.steps
    hmax = case.h.max()
    assert np.abs(h - case.h).max() <= 1e-12 * hmax
    om = oracle.Mesh(case.xy, case.tri)
    area = om.arrays()[2]
    c1 = gen.small(2)
    rc, st, h2, *_ = run_gpu(c1, "f64")
    area2 = oracle.Mesh(c1.xy, c1.tri).arrays()[2]
    m0, m1 = np.dot(c1.h, area2), np.dot(h2, area2)
    assert abs(m1 - m0) / m0 <= 1e-12


def test_tiny_meshes(gpu):
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float)
    one = gen.Case("one", xy[:3], np.array([[0, 1, 2]], np.int32), np.zeros(1), np.full(1, 0.03),
                   np.full(1, 0.7), np.zeros(1), np.zeros(1), 20)
    rc, st, h, hu, hv = run_gpu(one, "f64")
    assert rc == 0 and st["steps"] == 20
    assert abs(h[0] - 0.7) <= 1e-15 and abs(hu[0]) <= 1e-14 and abs(hv[0]) <= 1e-14
    two = gen.Case("two", xy, np.array([[0, 1, 2], [1, 3, 2]], np.int32), np.array([0.0, 0.1]),
                   np.full(2, 0.02), np.array([1.0, 0.2]), np.array([0.3, 0.0]),
                   np.array([0.0, -0.1]), 15)
    rc_o, *ora, _, st_o = run_oracle(two)
    rc_g, st_g, *g = run_gpu(two, "f64")
    assert rc_o == rc_g == 0
    assert max(errors(two, g, ora)) <= TOL_F64


@pytest.mark.parametrize("large", [False, True])
def test_dry_and_nonfinite_states_are_reported(gpu, large):
    """Up to 128 tiles the step folds its dt partials itself; the 40,000-cell mesh (157 tiles)
    merges them into atomic slots that a fold kernel reads."""
    import paper_1807_00672_amd as swe
    case = gen.dam_break(nx=200, ny=100, lx=40.0, ly=20.0) if large else gen.small(1)
    z = np.zeros(case.n_cells)
    dry = gen.Case("dry", case.xy, case.tri, z, z, z, z, z, 5)
    rc, st, *_ = run_gpu(dry, "f64")
    assert rc == swe.SWE_EDRY and st["steps"] == 0
    h = case.h.copy()
    h[1234] = np.nan
    bad = gen.Case("nan", case.xy, case.tri, z, z, h, z, z, 5)
    rc, st, *_ = run_gpu(bad, "f64")
    assert rc == swe.SWE_ENONFINITE
    h = case.h.copy()
    h[4321] = np.inf
    bad = gen.Case("inf", case.xy, case.tri, z, z, h, z, z, 5)
    rc, st, *_ = run_gpu(bad, "f32")
    assert rc == swe.SWE_ENONFINITE


def test_clamps_counted_through_the_atomic_slots(gpu):
    """A thin moving sheet stepped with a replayed dt about 2.5 times its CFL bound: a few cells
    drain below zero and are clamped.  On 40,000 cells (157 tiles) the step merges its clamp
    counts through the atomic slots; count, steps and fields against the oracle."""
    import copy
    case = copy.copy(gen.dam_break(nx=200, ny=100, lx=40.0, ly=20.0, h_right=0.0))
    case.h = np.full(case.n_cells, 0.01)
    case.hu = np.full(case.n_cells, 0.05)
    seq = np.full(6, 0.015)
    rc_o, *ora, dts, st_o = run_oracle(case, steps=6, dt_seq=seq)
    rc_g, st_g, *g = run_gpu(case, "f64", steps=6, dt_seq=seq)
    e = errors(case, g, ora)
    print(f"clamps {st_g['clamps']} vs {st_o['clamps']}; errors {e}")
    assert rc_o == 0 and rc_g == 0 and st_o["clamps"] > 0
    assert st_g["clamps"] == st_o["clamps"] and st_g["steps"] == st_o["steps"] == 6
    assert max(e) <= TOL_F64


@pytest.mark.parametrize("nx", [120, 360])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_three_mound_wet_dry_parity(gpu, dtype, nx):
    """11,520 cells (45 tiles: the step folds its dt partials itself) and 103,680 (405 tiles:
    atomic slots and a fold kernel), 600 steps with clamps and wet/dry fronts."""
    case = gen.three_mounds(nx=nx, ny=nx * 2 // 5)
    rc_o, *ora, dts, st_o = run_oracle(case if dtype == "f64" else float_rounded(case))
    rc_g, st_g, *g = run_gpu(case, dtype)
    assert rc_o == 0 and rc_g == 0 and st_g["steps"] == st_o["steps"] == case.steps
    hmax = np.abs(ora[0]).max()
    band = 0.0 if dtype == "f64" else TOL_F32 * hmax
    mism, exempt = mask_mismatch(case, g[0], ora[0], band=band)
    e = errors(case, g, ora)
    print(f"three mounds {dtype}: errors {e}, mask mismatches {mism} (exempt {exempt}), "
          f"clamps {st_g['clamps']} vs {st_o['clamps']}")
    assert mism == 0
    if dtype == "f64":
        assert max(e) <= TOL_F64 and st_g["clamps"] == st_o["clamps"]
    else:
        e_h, e_q = fp32_errors(case, g, ora)
        print(f"   h error {e_h:.2e} of max h, momentum error {e_q:.3f} of its bound")
        assert e_h <= TOL_F32 and e_q <= 1.0


def test_ritter_dry_bed_strip_parity(gpu):
    case = gen.strip(400, h_right=0.0)
    rc_o, *ora, dts, st_o = run_oracle(case, steps=100000, t_end=0.5)
    rc_g, st_g, *g = run_gpu(case, "f64", steps=5000, t_end=0.5)
    assert rc_o == 0 and rc_g == 0 and st_g["steps"] == st_o["steps"] and st_g["t"] == 0.5
    assert max(errors(case, g, ora)) <= TOL_F64
    assert np.array_equal(g[0] > case.h_dry, ora[0] > case.h_dry)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [2, 3, "ensemble"])
def test_quarter_turn_rotates_the_result_bitwise(gpu, k, dtype):
    """Every operation of the step is either unchanged by the turn (the same two products
    summed in the other order, lengths, |u|, areas) or odd in it (unit normals, momenta,
    divisions), so the turned mesh gives h unchanged and (hu, hv) -> (-hv, hu) bit for bit,
    although its cell order, tiles and halos all differ; "ensemble" has an inflow segment."""
    case = gen.ensemble_scenario(3, steps=60) if k == "ensemble" else gen.small(k)
    steps = 60
    turned = quarter_turn(case)
    rc, st, h, hu, hv = run_gpu(case, dtype, steps=steps)
    rc2, st2, h2, hu2, hv2 = run_gpu(turned, dtype, steps=steps)
    assert rc == rc2 == 0 and st["steps"] == st2["steps"] == steps and st["t"] == st2["t"]
    print(f"{case.name} {dtype}: {case.n_cells} cells, t = {st['t']:.6g}, "
          f"max |hu| {np.abs(hu).max():.3e}")
    assert np.abs(hu).max() > 0 and np.abs(hv).max() > 0
    assert np.array_equal(h2, h)
    assert np.array_equal(hu2, -hv)
    assert np.array_equal(hv2, hu)


@pytest.mark.parametrize("exact", [False, True])
def test_tile_node_lists_and_edge_vectors_give_the_same_bits(gpu, exact):
    """The FP64 tiled step forms each edge vector from its tile's node list by the mesh
    builder's own subtraction; without the node arrays it reads the stored edge vectors: the
    same run, bit for bit, in both FP64 math modes."""
    case = gen.small(3)
    m = gpu.Mesh(case.xy, case.tri)
    assert m.info.n_tile_nodes > 0 and m.dev.tile_nodes is not None

    def run():
        s = gpu.Solver(m, case.z, case.n, case.h, case.hu, case.hv, dtype="f64",
                       variant="tiled", exact=exact)
        rc, st = s.run(60)
        return rc, st, s.numpy_state()

    rc, st, (h, hu, hv) = run()
    m.dev.tile_node_off = m.dev.tile_nodes = m.dev.edge_nodes = None
    rc2, st2, (h2, hu2, hv2) = run()
    assert rc == rc2 == 0 and st["steps"] == st2["steps"] == 60 and st["t"] == st2["t"]
    assert np.array_equal(h, h2) and np.array_equal(hu, hu2) and np.array_equal(hv, hv2)
